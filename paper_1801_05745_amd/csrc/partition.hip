// Partitioned accumulation of the count maps (the keyed-sort form of the
// histogram of section 2.3 eq. (5)).
//
// Random 32-bit atomics into a GB-sized map run at a fixed ceiling on this GPU
// (about 2e10 per second), far below what the FP64 pixelisation delivers, so
// this path never updates the map once per instance.  Instead:
//   0. chunks: every wave of the key pass walks its own grid-stride sequence of
//      64-particle batches and stops before a batch once the key buffer could
//      not take the keys of one batch of every wave; it saves its position, and
//      the next chunk resumes there; the last chunk finishes every sequence
//      (no host synchronisation, no counting pass, no shared claim counter);
//   per chunk:
//   1. keys: the binning core emits key = b * npix + pix per instance into a
//      buffer (waves reserve 4096-slot chunks with one global atomic each) and,
//      with at most 256 level-1 buckets, counts each reservation's keys per
//      level-1 bucket in LDS, writing the counts when the reservation closes;
//   2. level-1 partition by key >> s1 (MSD radix step, <= 512 buckets; its
//      per-tile counts are sums of the reservations' counts when the key pass
//      took them, else a pass over the keys);
//   3. level 2, in place: each 32768-key super-tile of a level-1 bucket is
//      sorted by cell block (key >> 14) in LDS and written, as 16-bit cells,
//      at the positions it was read from (in a 16-bit view of the other key
//      buffer), with the start of every block's run in the tile;
//   4. accumulate: one workgroup per 16384-cell block counts the keys of its
//      runs (one per super-tile of its level-1 bucket) with LDS atomics and
//      adds the block into the map with coalesced 16-byte read-modify-writes
//      (blocks without keys are skipped).
// Level 1 works on super-tiles of 32768 keys: per-tile bucket counts, their
// exclusive scan per bucket (every tile's write offset), a scan of the bucket
// totals, then each super-tile ranked, sorted in LDS and written as contiguous
// runs, with no global atomics.  Level 2 needs no counting pass: its runs stay
// inside their super-tiles.  Integer counts make the result independent of
// every order involved.
#include "binning_core.hpp"

#include <algorithm>
#include <cmath>

namespace ufx {

constexpr int kBlockShift = 14;                  // cells per accumulation block: 2^14
constexpr int kBlockCells = 1 << kBlockShift;
constexpr int kSuper = 32768;                    // keys per partition super-tile
constexpr int kPartThreads = 256;
constexpr int kMaxBins = 512;                    // buckets per partition level
constexpr int kKeyWavesMax = 16 * kBinWaves;      // key-pass waves per compute unit, at most (per-wave state)
constexpr int kAccThreads = 512;

struct PartHeader {
    unsigned long long reserved;  // key slots reserved by the key pass of the current chunk
    unsigned int active;          // some wave has batches left: the current chunk runs
    unsigned int unfinished;      // waves that stopped on the margin in the current chunk
    unsigned long long pad[30];
};
static_assert(sizeof(PartHeader) == 256, "partition header is 256 bytes");

struct PartLayout {
    int s1;                 // level-1 shift
    int nb1, nb2;           // buckets per level
    int64_t nblk;           // cell blocks (nb1 * nb2 slots allocated)
    int kmax;               // chunk iterations launched
    unsigned long long cap; // key slots per buffer (multiple of kKeyChunk)
    unsigned long long margin;  // room a wave needs before it claims: every wave's worst-case claim
    unsigned long long budget;  // keys every chunk but the last processes, at least
    int64_t hist_rows;      // super-tile rows of the per-tile histogram
    bool counted;           // the key pass counts the level-1 buckets (nb1 <= kHistBins)
    size_t off_guard, off_hdr, off_wave, off_off1, off_tiles1, off_tot, off_thist, off_hrows, off_keysa, off_keysb,
        total;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int64_t kPartGuardEntries = 65536;

// Key slots a chunk keeps free: before each batch a wave checks that the slots
// reserved (as of its latest reservation) leave room for one batch of every
// wave (64 particles times the image bound, plus the up to kQueue queued images
// carried between batches, rounded up to whole reservations) and one more
// reservation; slack: one partly filled 4096-slot reservation per wave.  The
// key pass launches one resident round, so its waves are bounded by the
// workgroups per compute unit that the key kernels' occupancy allows.
static int key_wgs_per_cu();

static void claim_reserve(int64_t n, int img_bound, unsigned long long &margin, unsigned long long &slack) {
    const int64_t wgs = std::min<int64_t>((n + kBinBlock - 1) / kBinBlock, (int64_t)device_cus() * key_wgs_per_cu());
    const unsigned long long waves = (unsigned long long)std::max<int64_t>(wgs, 1) * kBinWaves;
    margin = waves * (64ull * (unsigned long long)img_bound + kQueue + kKeyChunk) + kKeyChunk;
    slack = waves * (unsigned long long)kKeyChunk;
}

// Layout for a call; want_keys = 0 means "as many as the bytes allow".
static bool plan_layout(PartLayout &L, int64_t n, int64_t ncells, int img_bound, size_t bytes, int64_t want_keys) {
    if (ncells <= 0 || ncells >= (int64_t)kNoKey) return false;
    int bits = 0;
    while (((int64_t)1 << bits) < ncells) ++bits;
    const int blk_bits = bits > kBlockShift ? bits - kBlockShift : 0;  // log2(#blocks), rounded up
    int b2 = blk_bits / 2;
    int b1 = blk_bits - b2;
    if (b1 > 9 || b2 > 9) return false;  // <= 512 buckets per level
    L.s1 = kBlockShift + b2;
    L.nb2 = 1 << b2;
    L.nb1 = (int)((ncells + ((int64_t)1 << L.s1) - 1) >> L.s1);
    L.nblk = (int64_t)L.nb1 * L.nb2;
    size_t o = 0;
    L.off_guard = o; o = align256(o + kGuardHeader + kPartGuardEntries * sizeof(GuardEntry));
    L.off_hdr = o; o = align256(o + sizeof(PartHeader));
    L.off_wave = o; o = align256(o + sizeof(int64_t) * (size_t)device_cus() * kKeyWavesMax);
    L.off_off1 = o; o = align256(o + sizeof(uint32_t) * (L.nb1 + 1));
    L.off_tiles1 = o; o = align256(o + sizeof(uint32_t) * (L.nb1 + 1));
    L.off_tot = o; o = align256(o + sizeof(uint32_t) * L.nb1);
    const size_t fixed_head = o;
    unsigned long long margin, slack;
    claim_reserve(n, img_bound, margin, slack);
    const int wide = std::max(L.nb1, L.nb2 + 1);  // level-1 counts, level-2 run starts (and the tile end)
    unsigned long long cap;
    if (want_keys > 0) {
        // two reservations of headroom: a layout re-derived from this one's byte count
        // (a plan's shared workspace) rounds its capacity down by up to one
        cap = std::max((unsigned long long)want_keys + margin + slack, 2 * (margin + slack)) + 3 * kKeyChunk;
    } else {
        // bytes = head + per-tile histogram (~ cap/kSuper rows) + per-reservation
        // level-1 counts + two key buffers
        const double per_key = 2.0 * sizeof(uint32_t) + (double)wide * sizeof(uint32_t) / kSuper +
                               (L.nb1 <= kHistBins ? (double)kHistBins * sizeof(uint16_t) / kKeyChunk : 0.0);
        // the rows beyond cap / kSuper: nb1 + 2, and up to 15 more that round to whole groups of 16
        const size_t extra = sizeof(uint32_t) * (size_t)wide * (L.nb1 + 2 + 15) + 4096;
        if (bytes < fixed_head + extra) return false;
        cap = (unsigned long long)((double)(bytes - fixed_head - extra) / per_key);
    }
    if (want_keys > 0) cap = (cap + kKeyChunk - 1) / kKeyChunk * kKeyChunk;  // whole reservations
    if (cap > 0xFFF00000ull) cap = 0xFFF00000ull;  // offsets are 32-bit
    cap = cap / kKeyChunk * kKeyChunk;
    // every chunk but the last must keep at least half of the buffer
    if (cap < 2 * (margin + slack) + kKeyChunk) return false;
    L.hist_rows = ((int64_t)(cap / kSuper) + L.nb1 + 2 + 15) / 16 * 16;  // whole groups of 16 tiles
    L.off_thist = o; o = align256(o + sizeof(uint32_t) * (size_t)wide * L.hist_rows);
    L.counted = L.nb1 <= kHistBins;
    L.off_hrows = o;
    if (L.counted) o = align256(o + sizeof(uint16_t) * (size_t)kHistBins * (size_t)(cap / kKeyChunk));
    const size_t fixed = o;
    L.cap = cap;
    L.margin = margin;
    L.budget = cap - margin - slack;
    L.off_keysa = fixed;
    L.off_keysb = align256(fixed + sizeof(uint32_t) * cap);
    L.total = align256(L.off_keysb + sizeof(uint32_t) * cap);
    // keys the set can produce at most; a chunk that stops on the margin has
    // processed at least `budget` of them, and the last chunk takes the rest
    const double est = (double)n * (double)img_bound;
    const int kmax_cap = 4096;
    if (est + (double)slack <= (double)cap) {
        L.kmax = 1;
    } else {
        const double k = std::ceil(est / (double)L.budget) + 1.0;
        L.kmax = (int)std::min<double>(k, (double)kmax_cap);
    }
    return true;
}

// Geometric bound on the images of one particle of [0, L)^3 that can reach the shell range.
static int image_bound(const BinCore &c, const double *e, int nb) {
    if (c.R == 0) return 1;
    const double o[3] = {c.ox, c.oy, c.oz};
    const double emin = e[0] * (1.0 - 1e-9), emax = e[nb] * (1.0 + 1e-9);
    int cnt = 0;
    for (int sx = -c.R; sx <= c.R; ++sx)
        for (int sy = -c.R; sy <= c.R; ++sy)
            for (int sz = -c.R; sz <= c.R; ++sz) {
                const int s[3] = {sx, sy, sz};
                double dmin = 0.0, dmax = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double lo = s[a] * c.L - o[a], hi = lo + c.L;
                    const double nearest = lo > 0.0 ? lo : (hi < 0.0 ? -hi : 0.0);
                    const double farthest = std::max(std::fabs(lo), std::fabs(hi));
                    dmin += nearest * nearest;
                    dmax += farthest * farthest;
                }
                if (std::sqrt(dmin) < emax && std::sqrt(dmax) >= emin) ++cnt;
            }
    return cnt > 0 ? cnt : 1;
}

// ------------------------------------------------------------------ kernels

// per-chunk reset of the key counter; chunk 0 runs when there are particles,
// a later chunk when some wave stopped on the margin in the previous one
__global__ void reset_chunk_kernel(PartHeader *hdr, int64_t n, int first) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr->reserved = 0ull;
        hdr->active = first ? (n > 0 ? 1u : 0u) : (hdr->unfinished > 0 ? 1u : 0u);
        hdr->unfinished = 0u;
    }
}

// 1. emit keys for the particles of the current chunk.  Wave v (of the same
// resident grid in every chunk) walks batches base_v, base_v + stride, ...;
// wave_pos[v] holds where it resumes.  Before a batch it checks that the slots
// reserved when it last reserved leave `margin` free (room for one batch of
// every wave), so a chunk never overflows its key buffer; the last chunk does not check and
// finishes every sequence (should its keys exceed the buffer, the rest are
// added by atomics and counted in n_fallback).
struct KeyParams {
    BinParams p;
    uint32_t *keys;
    unsigned long long cap;
    unsigned long long margin;
    PartHeader *hdr;
    int64_t *wave_pos;  // per wave: base of its next batch (-1: not started)
    uint16_t *hist_rows;  // per reservation: level-1 bucket counts (null: tile_hist counts them)
    int hist_shift;
    int last;
};

template <typename T>
__global__ __launch_bounds__(kBinBlock, 6) void keys_kernel(KeyParams kp) {
    const BinParams &p = kp.p;
    __shared__ EdgeLds E;
    __shared__ double qbuf[kBinWaves][3 * kQueue];
    __shared__ uint32_t hist_s[kBinWaves][kHistBins / 2];
    if (!kp.hdr->active) return;  // uniform: every wave finished in an earlier chunk
    load_edges(E, p.c, p.e);
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    if (kp.hist_rows) {
        reinterpret_cast<uint2 *>(hist_s[w])[lane] = make_uint2(0u, 0u);
        wave_lds_sync();
    }
    const int64_t wid = (int64_t)blockIdx.x * kBinWaves + w;
    const Shared sh = shared_of(p);
    LaneStats st;
    Emitter em{};
    em.keys = kp.keys;
    em.reserved = &kp.hdr->reserved;
    em.cap = kp.cap;
    em.hist = kp.hist_rows ? hist_s[w] : nullptr;
    em.hist_rows = kp.hist_rows;
    em.shift = kp.hist_shift;
    em.base = 0;
    em.fill = kKeyChunk + 1;  // no chunk held: the first key reserves one
    em.full = false;
    WaveQueue q{qbuf[w], 0, 0};
    const int64_t stride = (int64_t)gridDim.x * kBinBlock;
    const int64_t saved = kp.wave_pos[wid];
    const int64_t base = saved >= 0 ? saved : (int64_t)blockIdx.x * kBinBlock + w * 64;
    // The room check reads no memory: em.base, the reserved count the wave's
    // latest reservation returned, is a lower bound of the count at that moment.
    // Of the waves' last views before their last checks, the latest one covers
    // every reservation made before any of those checks, and each wave adds at
    // most one batch after its last check: the margin bounds the total.
    const unsigned long long limit = kp.cap - kp.margin;
    const bool last = kp.last != 0;
    auto full = [&]() { return !last && em.base > limit; };
    int64_t next = base;
    if (base < p.c.n && !full()) next = bin_wave_range<T, kEmit>(p.c, sh, E, base, p.c.n, stride, q, st, em, full);
    drain_queue<kEmit>(p.c, sh, E, q, st, em);
    close_emitter(em);
    if (lane == 0) {
        kp.wave_pos[wid] = next;
        if (next < p.c.n) atomicAdd(&kp.hdr->unfinished, 1u);
    }
    flush_stats(p.status, st);
}

static int key_wgs_per_cu() {
    static int v = 0;
    if (!v) {
        int a = 0, b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, keys_kernel<float>, kBinBlock, 0) != hipSuccess) a = 16;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, keys_kernel<double>, kBinBlock, 0) != hipSuccess) b = 16;
        v = std::min(std::max(std::max(a, b), 1), kKeyWavesMax / kBinWaves);
    }
    return v;
}

// Partition steps.  Level 1: one segment keys[0, reserved) (with sentinels),
// bucket = key >> shift, cut into super-tiles of kSuper keys; the per-tile
// bucket counts (l1_rows or tile_hist) are scanned per bucket by bucket_scan
// into per-tile write offsets (and bucket totals), bucket_base scans the
// totals, and scatter writes every key at base[bucket] + offset[bucket][tile]
// + its rank inside the super-tile, sorting each super-tile in LDS so that each
// bucket's keys leave as contiguous runs.  Level 2: segment s = level-1 bucket
// s (keys with key >> s1 == s), bucket = (key >> shift) - s * nbins, the global
// bucket s * nbins + b being the cell block; each super-tile of a segment is
// sorted in place and records where each bucket's run starts.  No global
// atomics; ranks inside a sub-tile come from LDS atomics.
struct PartStep {
    const uint32_t *in;
    uint32_t *out;              // level 1: full keys
    uint16_t *out16;            // level 2: the key's cell inside its block (the block is the position)
    int level;
    int nseg;
    const uint32_t *seg_off;    // level 2: [nseg + 1] segment starts in `in`
    const uint32_t *seg_tiles;  // level 2: [nseg + 1] first super-tile of each segment
    const PartHeader *hdr;      // level 1: reserved slots
    unsigned long long cap;
    int shift, nbins;
    uint32_t *tile_hist;        // level 1: [nbins][max_tiles] counts, then offsets inside the bucket;
                                // level 2: [ntiles][nbins + 1] run starts inside the tile, then its key count
    uint32_t *bucket_tot;       // level 1: [nbins]
    uint32_t *bucket_base;      // level 1: [nbins + 1] exclusive scan of bucket_tot
    int64_t max_tiles;          // tiles allocated in tile_hist
};

__device__ __forceinline__ int64_t step_total(const PartStep &ps) {
    unsigned long long total = ps.hdr->reserved;
    return (int64_t)(total > ps.cap ? ps.cap : total);
}

__device__ __forceinline__ int64_t step_tiles(const PartStep &ps) {
    if (ps.level == 1) return (step_total(ps) + kSuper - 1) / kSuper;
    return ps.seg_tiles[ps.nseg];
}

__device__ __forceinline__ void seg_range(const PartStep &ps, int64_t t, int &seg, int64_t &lo, int64_t &hi) {
    if (ps.level == 1) {
        const int64_t total = step_total(ps);
        seg = 0;
        lo = t * kSuper;
        hi = lo + kSuper < total ? lo + kSuper : total;
        return;
    }
    int a = 0, b = ps.nseg;  // largest s with seg_tiles[s] <= t
    while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (ps.seg_tiles[mid] <= t) a = mid; else b = mid;
    }
    seg = a;
    lo = (int64_t)ps.seg_off[a] + (t - ps.seg_tiles[a]) * kSuper;
    hi = lo + kSuper < (int64_t)ps.seg_off[a + 1] ? lo + kSuper : (int64_t)ps.seg_off[a + 1];
}

// Workgroup barrier that orders LDS only.  __syncthreads() also makes every
// thread wait for its own outstanding global stores, which the partition
// kernels never need: no thread reads global memory that another thread of the
// workgroup wrote during the launch.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS counting by a wave, one bucket per lane (valid lanes only; all 64 lanes
// call it).  When every valid lane holds the same bucket, as keys of spatially
// ordered particles mostly do, one atomic adds the wave's count instead of 64
// atomics on one address, which the LDS would serialise.
__device__ __forceinline__ void wave_count(uint32_t *h, uint32_t bin, bool valid) {
    const unsigned long long vm = wave_ballot(valid);
    if (vm == 0ull) return;
    const int first = __builtin_ctzll(vm);
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)bin, first);
    if (wave_ballot(valid && bin == b0) == vm) {
        if ((int)(threadIdx.x & 63) == first) atomicAdd(&h[b0], (uint32_t)__popcll(vm));
    } else if (valid) {
        atomicAdd(&h[bin], 1u);
    }
}

// per-super-tile bucket counts (wave-private LDS histograms, summed); 16 loads
// in flight per thread
constexpr int kHistUnroll = 16;
__global__ __launch_bounds__(kPartThreads) void tile_hist_kernel(PartStep ps) {
    constexpr int kW = kPartThreads / 64;
    __shared__ uint32_t wh[kW][kMaxBins];
    if (!ps.hdr->active) return;
    const int tid = threadIdx.x, w = tid >> 6;
    const int64_t ntiles = step_tiles(ps);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int seg;
        int64_t lo, hi;
        seg_range(ps, t, seg, lo, hi);
        const uint32_t bin0 = (uint32_t)seg * (uint32_t)ps.nbins;
        for (int b = tid; b < ps.nbins; b += kPartThreads)
            for (int k = 0; k < kW; ++k) wh[k][b] = 0u;
        lds_barrier();
        for (int64_t base = lo; base < hi; base += (int64_t)kPartThreads * kHistUnroll) {
            uint32_t kk[kHistUnroll];
#pragma unroll
            for (int u = 0; u < kHistUnroll; ++u) {
                const int64_t i = base + (int64_t)u * kPartThreads + tid;
                kk[u] = i < hi ? ps.in[i] : kNoKey;
            }
#pragma unroll
            for (int u = 0; u < kHistUnroll; ++u)
                wave_count(wh[w], (kk[u] >> ps.shift) - bin0, kk[u] != kNoKey);
        }
        lds_barrier();
        for (int b = tid; b < ps.nbins; b += kPartThreads) {
            uint32_t c = 0;
            for (int k = 0; k < kW; ++k) c += wh[k][b];
            ps.tile_hist[b * ps.max_tiles + t] = c;
        }
        lds_barrier();
    }
}

// Level-1 bucket counts per super-tile from the key pass's per-reservation
// counts (super-tile t holds reservations t * kSuper / kKeyChunk onwards): the
// tile_hist of level 1 without reading the keys.  A workgroup takes kRowGroup
// consecutive tiles, so that each bucket's counts leave as 16-byte stores
// (max_tiles is a multiple of kRowGroup; counts past the last tile are zero).
static_assert(kSuper % kKeyChunk == 0, "super-tiles are whole reservations");
constexpr int kRowGroup = 16;
__global__ __launch_bounds__(kHistBins) void l1_rows_kernel(PartStep ps, const uint16_t *hrows) {
    constexpr int kPerTile = kSuper / kKeyChunk;
    if (!ps.hdr->active) return;
    const int64_t nres = step_total(ps) / kKeyChunk;  // reserved slots come in whole reservations
    const int64_t ngroups = (step_tiles(ps) + kRowGroup - 1) / kRowGroup;
    const int b = threadIdx.x;
    for (int64_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
        uint32_t c[kRowGroup];
#pragma unroll
        for (int i = 0; i < kRowGroup; ++i) {
            const int64_t r0 = (gi * kRowGroup + i) * kPerTile;
            const int64_t r1 = r0 + kPerTile < nres ? r0 + kPerTile : nres;
            c[i] = 0u;
            for (int64_t r = r0; r < r1; ++r) c[i] += hrows[r * kHistBins + b];
        }
        if (b < ps.nbins) {
            uint4 *dst = reinterpret_cast<uint4 *>(ps.tile_hist + b * ps.max_tiles + gi * kRowGroup);
#pragma unroll
            for (int i = 0; i < kRowGroup / 4; ++i) dst[i] = make_uint4(c[4 * i], c[4 * i + 1], c[4 * i + 2], c[4 * i + 3]);
        }
    }
}

// level 1, one workgroup per bucket b: exclusive offsets of the bucket's keys
// over the super-tiles, and the bucket total
__global__ __launch_bounds__(256) void bucket_scan_kernel(PartStep ps) {
    __shared__ uint32_t wsum[4];
    if (!ps.hdr->active) return;
    const int64_t g = blockIdx.x;
    const int b = (int)g;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t t0 = 0, t1 = step_tiles(ps);
    uint32_t *col = ps.tile_hist + b * ps.max_tiles;  // the bucket's counts over the tiles, contiguous
    uint32_t carry = 0;
    for (int64_t base = t0; base < t1; base += 256) {
        const int64_t t = base + threadIdx.x;
        const uint32_t v = t < t1 ? col[t] : 0u;
        uint32_t x = v;  // inclusive scan inside the wave
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int k = 0; k < w; ++k) before += wsum[k];
        if (t < t1) col[t] = before + x - v;
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) ps.bucket_tot[g] = carry;
}

// exclusive scan of the level-1 bucket totals (one workgroup, running carry),
// and the first super-tile of every level-2 segment.  Each thread scans kPer
// consecutive totals serially; the thread sums are scanned across the wave
// with shuffles and across the 16 waves through LDS: two barriers per
// 1024 * kPer totals.
__global__ __launch_bounds__(1024) void bucket_base_kernel(const uint32_t *tot, int64_t nbkt, uint32_t *base,
                                                           uint32_t *tiles, const PartHeader *hdr) {
    constexpr int kPer = 8;
    constexpr int kW = 1024 / 64;
    __shared__ unsigned long long wh[kW], wt[kW];
    if (!hdr->active) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    unsigned long long carry = 0, carry_t = 0;  // uniform over the workgroup
    for (int64_t s = 0; s < nbkt; s += 1024 * kPer) {
        const int64_t i0 = s + (int64_t)tid * kPer;
        uint32_t h[kPer];
        unsigned long long sh = 0, st = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            h[u] = i0 + u < nbkt ? tot[i0 + u] : 0u;
            sh += h[u];
            st += (h[u] + kSuper - 1) / kSuper;
        }
        unsigned long long xh = sh, xt = st;  // inclusive scan over the wave
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long yh = __shfl_up(xh, off, 64), yt = __shfl_up(xt, off, 64);
            if (lane >= off) {
                xh += yh;
                xt += yt;
            }
        }
        if (lane == 63) {
            wh[w] = xh;
            wt[w] = xt;
        }
        __syncthreads();
        unsigned long long ph = carry + xh - sh, pt = carry_t + xt - st;
        unsigned long long seg_h = 0, seg_t = 0;
        for (int k = 0; k < kW; ++k) {
            if (k < w) {
                ph += wh[k];
                pt += wt[k];
            }
            seg_h += wh[k];
            seg_t += wt[k];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (i0 + u < nbkt) {
                base[i0 + u] = (uint32_t)ph;
                if (tiles) tiles[i0 + u] = (uint32_t)pt;
            }
            ph += h[u];
            pt += (h[u] + kSuper - 1) / kSuper;
        }
        carry += seg_h;
        carry_t += seg_t;
        __syncthreads();  // wh/wt are rewritten by the next segment
    }
    if (tid == 0) {
        base[nbkt] = (uint32_t)carry;
        if (tiles) tiles[nbkt] = (uint32_t)carry_t;
    }
}


// scatter: per sub-tile (the whole 32768-key super-tile: 128 KiB of LDS, one
// workgroup per compute unit; longer runs per bucket than 8192-key sub-tiles,
// about 10 % less time), ranks from LDS atomics on the bucket counts,
// a bucket-order scan, an LDS sort, then contiguous runs written at base + tile
// offset + running count.  Key order inside a bucket is irrelevant to the
// counts, so the nondeterministic order of the atomics is harmless.
// kInPlace (level 2): the sorted tile is written at the positions it was read
// from (16-bit cells, in out16) and the tile's row of tile_hist receives its
// bucket starts.  Each bucket's
// count is split over 2^ss lane classes (lane mod 4, fewer when the buckets are
// many: one counter per thread in the scan): the keys of a wave that share a
// bucket, as spatially ordered particles' keys do, then contend on four LDS
// counters rather than one (partition 42 % faster on cell-ordered particles,
// 2 % slower on shuffled ones), and a bucket's classes stay adjacent in the
// sorted order.
constexpr int kScatThreads = 1024;  // 16 waves per compute unit: about 12 % faster than 512
constexpr int kSub = kSuper;
template <typename OutT, bool kInPlace = false>
__global__ __launch_bounds__(kScatThreads, 1) void scatter_kernel(PartStep ps) {
    static_assert(sizeof(OutT) == 4 || sizeof(OutT) == 2, "full keys or 16-bit cell indices");
    static_assert(!kInPlace || (kSub == kSuper && sizeof(OutT) == 2), "an in-place tile is one sub-tile of cells");
    static_assert(kBlockShift <= 16, "a cell index inside a block fits 16 bits");
    constexpr int kW = kScatThreads / 64;
    constexpr int kPer = kSub / kScatThreads;  // keys per thread per sub-tile
    static_assert(kMaxBins <= kScatThreads, "one counter per thread in the scan");
    static_assert(kSub <= 65536 && kScatThreads <= 65536, "counter and rank packed in 16-bit halves");
    __shared__ uint32_t cnt[kScatThreads];       // keys per (bucket, lane class) in the sub-tile
    __shared__ uint32_t gbase[kMaxBins];         // global start of this super-tile's run per bucket
    __shared__ uint32_t run[kMaxBins];           // keys of the bucket written by earlier sub-tiles
    __shared__ uint32_t soff[kScatThreads + 1];  // (bucket, class) start inside the sorted sub-tile
    __shared__ uint32_t dst[kMaxBins];           // global position of sorted slot 0 of the bucket (mod 2^32)
    __shared__ uint32_t skeys[kSub];
    __shared__ uint32_t wsum[kW];
    if (!ps.hdr->active) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    int ss = 0;  // lane classes per bucket: 2^ss
    while (ss < 2 && (ps.nbins << (ss + 1)) <= kScatThreads) ++ss;
    const int nsub = ps.nbins << ss;
    const uint32_t cls = (uint32_t)lane & ((1u << ss) - 1u);
    const int64_t ntiles = step_tiles(ps);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int seg;
        int64_t lo, hi;
        seg_range(ps, t, seg, lo, hi);
        const uint32_t bin0 = (uint32_t)seg * (uint32_t)ps.nbins;
        if (!kInPlace && tid < ps.nbins) {
            gbase[tid] = ps.bucket_base[bin0 + tid] + ps.tile_hist[tid * ps.max_tiles + t];
            run[tid] = 0u;
        }
        for (int64_t sub = lo; sub < hi; sub += kSub) {
            const int64_t shi = sub + kSub < hi ? sub + kSub : hi;
            if (tid < nsub) cnt[tid] = 0u;
            lds_barrier();                                                  // 1
            // rank pass; rk = counter << 16 | rank at the counter, ~0 for no key.
            // Loads are unconditional at clamped indices so that all of them are in
            // flight together; a wave with no keys in the sub-tile skips them.
            const int64_t w0 = sub + (int64_t)w * kPer * 64;  // wave w: keys [w0, w0 + kPer 64)
            const int rem = (int)(shi - w0 < 0 ? 0 : (shi - w0 < kPer * 64 ? shi - w0 : kPer * 64));
            const uint32_t *src = ps.in + w0;
            uint32_t kv[kPer], rk[kPer];
            if (rem > 0) {
#pragma unroll
                for (int u = 0; u < kPer; ++u) kv[u] = src[min(u * 64 + lane, rem - 1)];
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    const bool valid = u * 64 + lane < rem && kv[u] != kNoKey;
                    const uint32_t sb = ((kv[u] >> ps.shift) - bin0) << ss | cls;
                    rk[u] = valid ? sb << 16 | atomicAdd(&cnt[sb], 1u) : ~0u;
                }
            }
            lds_barrier();                                                  // 2
            const uint32_t c = tid < nsub ? cnt[tid] : 0u;
            uint32_t x = c;  // inclusive scan within the wave, counter order = thread order
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off, 64);
                if (lane >= off) x += y;
            }
            if (lane == 63) wsum[w] = x;
            lds_barrier();                                                  // 3
            uint32_t acc = x - c;
            for (int k = 0; k < w; ++k) acc += wsum[k];
            if (tid < nsub) soff[tid] = acc;
            if (tid == kScatThreads - 1) soff[nsub] = acc + c;
            lds_barrier();                                                  // 4
            // per bucket: its first class's start; the keys placed in counter order
            if (tid <= ps.nbins) {
                const uint32_t start = soff[tid << ss];  // soff[nsub]: the sub-tile's key count
                if (!kInPlace && tid < ps.nbins) dst[tid] = gbase[tid] + run[tid] - start;
                if (kInPlace) ps.tile_hist[t * (int64_t)(ps.nbins + 1) + tid] = start;
            }
            if (rem > 0) {
#pragma unroll
                for (int u = 0; u < kPer; ++u)
                    if (rk[u] != ~0u) skeys[soff[rk[u] >> 16] + (rk[u] & 0xFFFFu)] = kv[u];
            }
            lds_barrier();                                                  // 5
            const uint32_t nv = soff[nsub];
            if (nv > 0) {
                // unrolled, reads at clamped indices, so that the LDS reads overlap
#pragma unroll 8
                for (int j = 0; j < kPer; ++j) {
                    const uint32_t sidx = (uint32_t)(j * kScatThreads + tid);
                    const uint32_t key = skeys[min(sidx, nv - 1u)];
                    const uint32_t pos = (kInPlace ? (uint32_t)sub : dst[(key >> ps.shift) - bin0]) + sidx;
                    if (sidx < nv) {
                        if constexpr (sizeof(OutT) == 4)
                            ps.out[pos] = key;
                        else
                            ps.out16[pos] = (uint16_t)(key & (kBlockCells - 1));
                    }
                }
            }
            lds_barrier();                                                  // 6
            if (!kInPlace && tid < ps.nbins) run[tid] += soff[(tid + 1) << ss] - soff[tid << ss];
        }
    }
}

// 5. one workgroup per cell block g = seg * nbins + b of level 2: the block's
// keys are one run in each super-tile of level-1 bucket seg (run starts in the
// tile's row of tile_hist).  Up to kAccThreads runs at a time are listed in LDS;
// kLanes lanes read one run in aligned 16-byte words of 8 cells (kLanes near a
// quarter of the mean run, kSuper / nbins cells, so one word per lane covers
// most runs), a wave reads kRows * 64 / kLanes runs at once (kRows loads per
// lane in flight), and the cells of each word that lie inside the run go into
// the LDS histogram; finally counts += histogram.
template <int kLanes>
__global__ __launch_bounds__(kAccThreads) void accumulate_kernel(PartStep ps, const uint16_t *cells, int64_t ncells,
                                                                 uint32_t *counts) {
    static_assert(kLanes == 16 || kLanes == 32 || kLanes == 64, "lanes per run divide the wave");
    constexpr int kW = kAccThreads / 64;
    constexpr int kRows = kLanes == 64 ? 8 : 4;  // within 128 registers: two workgroups per compute unit
    constexpr int kRunsPerWave = kRows * 64 / kLanes;
    __shared__ uint32_t h[kBlockCells];
    __shared__ uint32_t rlo[kAccThreads], rhi[kAccThreads];  // the pass's runs: cells [lo, hi)
    __shared__ uint32_t nkeys;
    if (!ps.hdr->active) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int slot = lane / kLanes, sub = lane % kLanes;  // run slot in a row, lane inside the run
    const uint4 *words = reinterpret_cast<const uint4 *>(cells);  // the buffer is 256-byte aligned
    const int64_t stride = ps.nbins + 1;
    const int64_t nblk = (int64_t)ps.nseg * ps.nbins;
    for (int64_t g = blockIdx.x; g < nblk; g += gridDim.x) {
        const int seg = (int)(g / ps.nbins), b = (int)(g % ps.nbins);
        const int64_t t0 = ps.seg_tiles[seg], t1 = ps.seg_tiles[seg + 1];
        if (t0 == t1) continue;  // uniform over the block: an empty level-1 bucket
        for (int j = threadIdx.x; j < kBlockCells; j += kAccThreads) h[j] = 0u;
        if (threadIdx.x == 0) nkeys = 0u;
        const uint32_t sbase = ps.seg_off[seg];
        uint32_t mine = 0;  // cells this thread listed
        for (int64_t tb = t0; tb < t1; tb += kAccThreads) {
            const int64_t tt = tb + threadIdx.x;
            uint32_t lo = 0u, hi = 0u;
            if (tt < t1) {
                const uint32_t *row = ps.tile_hist + tt * stride;
                const uint32_t base = sbase + (uint32_t)(tt - t0) * (uint32_t)kSuper;
                lo = base + row[b];
                hi = base + row[b + 1];
            }
            rlo[threadIdx.x] = lo;
            rhi[threadIdx.x] = hi;
            mine += hi - lo;
            lds_barrier();  // the list is complete (and, on the first pass, h is clear)
            const int nr = (int)(t1 - tb < kAccThreads ? t1 - tb : kAccThreads);
            for (int r0 = w * kRunsPerWave; r0 < nr; r0 += kW * kRunsPerWave) {
                // this lane's run in row p: r0 + p * (64 / kLanes) + slot
                uint32_t clo[kRows], chi[kRows], w0[kRows], nw[kRows], longest = 0;
#pragma unroll
                for (int p = 0; p < kRows; ++p) {
                    const int r = r0 + p * (64 / kLanes) + slot;
                    clo[p] = r < nr ? rlo[r] : 0u;
                    chi[p] = r < nr ? rhi[r] : 0u;
                    w0[p] = clo[p] >> 3;
                    nw[p] = chi[p] > clo[p] ? ((chi[p] + 7u) >> 3) - w0[p] : 0u;
                    longest = max(longest, nw[p]);
                }
                for (uint32_t k = 0; wave_ballot(k < longest) != 0ull; k += kLanes) {
                    uint4 v[kRows];
#pragma unroll
                    for (int p = 0; p < kRows; ++p) {
                        const uint32_t kk = k + (uint32_t)sub;
                        v[p] = kk < nw[p] ? words[w0[p] + kk] : make_uint4(0u, 0u, 0u, 0u);
                    }
#pragma unroll
                    for (int p = 0; p < kRows; ++p) {
                        // cells [e0, e0 + 8) of the word; those in [clo, chi) count
                        const uint32_t e0 = (w0[p] + k + (uint32_t)sub) * 8u;
                        const uint32_t qlo = clo[p] > e0 ? clo[p] - e0 : 0u;
                        const uint32_t qhi = chi[p] > e0 ? min(chi[p] - e0, 8u) : 0u;
                        const uint32_t m = ((1u << qhi) - 1u) & ~((1u << qlo) - 1u);
                        const uint32_t x[4] = {v[p].x, v[p].y, v[p].z, v[p].w};
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (m & (1u << q)) atomicAdd(&h[(x[q >> 1] >> (16 * (q & 1))) & 0xFFFFu], 1u);
                    }
                }
            }
            lds_barrier();  // every wave is done with the list before the next pass rewrites it
        }
        if (mine) atomicAdd(&nkeys, mine);
        lds_barrier();
        if (nkeys == 0u) continue;  // uniform: a block without keys keeps its counts untouched
        const int64_t c0 = g * kBlockCells;
        const int64_t cn = c0 + kBlockCells < ncells ? kBlockCells : ncells - c0;  // multiple of 4
        uint4 *dst = reinterpret_cast<uint4 *>(counts + c0);
        const int nq = (int)(cn / 4);
        // the block's 16-byte words, all read before any is written back
        constexpr int kPerThread = kBlockCells / 4 / kAccThreads;
        uint4 v[kPerThread];
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            const int j = u * kAccThreads + threadIdx.x;
            if (j < nq) v[u] = dst[j];
        }
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            const int j = u * kAccThreads + threadIdx.x;
            if (j < nq) {
                v[u].x += h[4 * j];
                v[u].y += h[4 * j + 1];
                v[u].z += h[4 * j + 2];
                v[u].w += h[4 * j + 3];
                dst[j] = v[u];
            }
        }
        lds_barrier();
    }
}

// guarded instances listed by the key passes
__global__ __launch_bounds__(256) void part_guarded_kernel(BinParams p) {
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

template <typename T>
__global__ __launch_bounds__(kBinBlock) void part_rescue_kernel(BinParams p) {
    if (p.guard->overflow == 0u) return;
    __shared__ EdgeLds E;
    __shared__ double qbuf[kBinWaves][3 * kQueue];
    __shared__ double radii[UFALCON_MAX_SHELLS + 1];
    load_edges(E, p.c, p.e, radii);
    const int w = threadIdx.x >> 6;
    const Shared sh = shared_of(p);
    LaneStats st;
    Emitter em{};
    WaveQueue q{qbuf[w], 0, 0};
    bin_wave_range<T, kRescue>(p.c, sh, E, (int64_t)blockIdx.x * kBinBlock + w * 64, p.c.n,
                               (int64_t)gridDim.x * kBinBlock, q, st, em);
    drain_queue<kRescue>(p.c, sh, E, q, st, em);
    flush_stats(p.status, st);
}

__global__ void part_guard_reset_kernel(GuardList *g, PartHeader *hdr, int64_t *wave_pos, int64_t nwaves) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        g->count = 0u;
        g->overflow = 0u;
        hdr->unfinished = 0u;
    }
    if (i < nwaves) wave_pos[i] = -1;
}

template <typename T>
int launch_partitioned(BinParams p, const PartLayout &L, int img_bound, char *ws, hipStream_t s,
                       ufalcon_phase_timer *timer, const PartHooks *hooks) {
    GuardList *guard = reinterpret_cast<GuardList *>(ws + L.off_guard);
    PartHeader *hdr = reinterpret_cast<PartHeader *>(ws + L.off_hdr);
    uint32_t *off1 = reinterpret_cast<uint32_t *>(ws + L.off_off1);
    uint32_t *tiles1 = reinterpret_cast<uint32_t *>(ws + L.off_tiles1);
    uint32_t *tot = reinterpret_cast<uint32_t *>(ws + L.off_tot);
    uint32_t *thist = reinterpret_cast<uint32_t *>(ws + L.off_thist);
    uint32_t *keysa = reinterpret_cast<uint32_t *>(ws + L.off_keysa);
    uint32_t *keysb = reinterpret_cast<uint32_t *>(ws + L.off_keysb);
    p.guard = guard;
    p.guard_cap = kPartGuardEntries;
    const int64_t ncells = (int64_t)p.c.nb * p.npix;
    const unsigned cus = (unsigned)device_cus();

    int64_t *wave_pos = reinterpret_cast<int64_t *>(ws + L.off_wave);
    // one resident round of waves, the same in every chunk (wave v resumes its own sequence)
    const unsigned key_grid = blocks_for(p.c.n, kBinBlock, resident_grid(keys_kernel<T>, kBinBlock, cus));
    const int64_t nwaves = (int64_t)key_grid * kBinWaves;
    if (nwaves > (int64_t)cus * kKeyWavesMax) return UFALCON_EWORKSPACE;  // never: the grid is one resident round

    timer_start(timer, s);
    hipLaunchKernelGGL(part_guard_reset_kernel, dim3(blocks_for(nwaves, 256)), dim3(256), 0, s, guard, hdr, wave_pos,
                       nwaves);
    timer_mark(timer, UFALCON_PHASE_SETUP, s);

    KeyParams kp;
    kp.p = p;
    kp.keys = keysa;
    kp.cap = L.cap;
    kp.hdr = hdr;
    kp.wave_pos = wave_pos;
    kp.hist_rows = L.counted ? reinterpret_cast<uint16_t *>(ws + L.off_hrows) : nullptr;
    kp.hist_shift = L.s1;

    PartStep l1{};
    l1.in = keysa;
    l1.out = keysb;
    l1.level = 1;
    l1.nseg = 1;
    l1.hdr = hdr;
    l1.cap = L.cap;
    l1.shift = L.s1;
    l1.nbins = L.nb1;
    l1.tile_hist = thist;
    l1.bucket_tot = tot;
    l1.bucket_base = off1;
    l1.max_tiles = L.hist_rows;

    PartStep l2 = l1;
    l2.in = keysb;
    l2.out = nullptr;
    l2.out16 = reinterpret_cast<uint16_t *>(keysa);
    l2.level = 2;
    l2.nseg = L.nb1;
    l2.seg_off = off1;
    l2.seg_tiles = tiles1;
    l2.shift = kBlockShift;
    l2.nbins = L.nb2;
    l2.bucket_base = nullptr;  // in place: runs stay inside their super-tiles
    l2.bucket_tot = nullptr;

    const unsigned hist_grid = resident_grid(tile_hist_kernel, kPartThreads, cus);
    const unsigned scat_grid = resident_grid(scatter_kernel<uint32_t>, kScatThreads, cus);
    // lanes per run near a quarter of the mean run (kSuper / nb2 cells): about one 8-cell word per lane
    const int mean_run = kSuper / L.nb2;
    auto acc = mean_run <= 64 ? accumulate_kernel<16> : (mean_run <= 128 ? accumulate_kernel<32> : accumulate_kernel<64>);
    const unsigned acc_grid = resident_grid(acc, kAccThreads, cus);
    for (int k = 0; k < L.kmax; ++k) {
        hipLaunchKernelGGL(reset_chunk_kernel, dim3(1), dim3(64), 0, s, hdr, p.c.n, k == 0 ? 1 : 0);
        kp.margin = L.margin;
        kp.last = k + 1 == L.kmax ? 1 : 0;  // the last chunk takes every particle left
        if (k == 0 && hooks && hooks->wait_keys) UFX_HIP_CHECK(hipStreamWaitEvent(s, hooks->wait_keys, 0));
        hipLaunchKernelGGL((keys_kernel<T>), dim3(key_grid), dim3(kBinBlock), 0, s, kp);
        if (k == 0 && hooks && hooks->done_keys) UFX_HIP_CHECK(hipEventRecord(hooks->done_keys, s));
        timer_mark(timer, UFALCON_PHASE_DECIDE, s);
        // level 1: by key >> s1 (the key pass counted the buckets when there are few enough)
        if (kp.hist_rows)
            hipLaunchKernelGGL(l1_rows_kernel, dim3(hist_grid), dim3(kHistBins), 0, s, l1,
                               (const uint16_t *)kp.hist_rows);
        else
            hipLaunchKernelGGL(tile_hist_kernel, dim3(hist_grid), dim3(kPartThreads), 0, s, l1);
        hipLaunchKernelGGL(bucket_scan_kernel, dim3((unsigned)L.nb1), dim3(256), 0, s, l1);
        hipLaunchKernelGGL(bucket_base_kernel, dim3(1), dim3(1024), 0, s, tot, (int64_t)L.nb1, off1, tiles1, hdr);
        hipLaunchKernelGGL(scatter_kernel<uint32_t>, dim3(scat_grid), dim3(kScatThreads), 0, s, l1);
        // level 2: every super-tile of a level-1 bucket sorted by cell block, in place
        hipLaunchKernelGGL((scatter_kernel<uint16_t, true>), dim3(scat_grid), dim3(kScatThreads), 0, s, l2);
        timer_mark(timer, UFALCON_PHASE_PARTITION, s);
        hipLaunchKernelGGL(acc, dim3((unsigned)std::min<int64_t>(L.nblk, acc_grid)), dim3(kAccThreads), 0, s, l2,
                           reinterpret_cast<const uint16_t *>(keysa), ncells, p.c.counts);
        timer_mark(timer, UFALCON_PHASE_ACCUMULATE, s);
        if (k == 0 && fault_injected("partition_chunk")) {  // tests of error handling; never inside a capture
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) return UFALCON_EINJECTED;
        }
    }
    hipLaunchKernelGGL(part_guarded_kernel, dim3(64), dim3(256), 0, s, p);
    hipLaunchKernelGGL((part_rescue_kernel<T>), dim3(key_grid), dim3(kBinBlock), 0, s, p);
    timer_mark(timer, UFALCON_PHASE_EXACT, s);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

// Entry from ufalcon_bin_shells: returns 1 if the partitioned path was taken.
int try_partitioned(BinParams &p, int dtype, void *workspace, size_t bytes, hipStream_t s, int *rc,
                    ufalcon_phase_timer *timer, const PartHooks *hooks) {
    const int64_t ncells = (int64_t)p.c.nb * p.npix;
    if ((uintptr_t)p.c.counts & 15u) return 0;  // the block update uses 16-byte accesses
    PartLayout L;
    const int img = image_bound(p.c, p.e, p.c.nb);
    if (!plan_layout(L, p.c.n, ncells, img, bytes, 0)) return 0;
    if (L.total > bytes) return 0;
    char *ws = static_cast<char *>(workspace);
    *rc = dtype == UFALCON_F32 ? launch_partitioned<float>(p, L, img, ws, s, timer, hooks)
                               : launch_partitioned<double>(p, L, img, ws, s, timer, hooks);
    return 1;
}

// Workspace for one particle set with keys for all its images in one chunk (capped at 32-bit offsets).
size_t partitioned_size_for(const BinParams &p) {
    const int img = image_bound(p.c, p.e, p.c.nb);
    const double want = std::min<double>((double)p.c.n * img, 4.0e9);
    PartLayout L;
    if (!plan_layout(L, p.c.n, (int64_t)p.c.nb * p.npix, img, 0, std::max<int64_t>((int64_t)want, 1))) return 0;
    return L.total;
}

size_t partitioned_workspace_size(int64_t n, int64_t ncells, int img_bound, int64_t max_keys) {
    PartLayout L;
    if (!plan_layout(L, n, ncells, img_bound, 0, max_keys)) return 0;
    return L.total;
}

}  // namespace ufx

using namespace ufx;

extern "C" int64_t ufalcon_bin_shells_partition_capacity(int64_t n, int32_t n_rep, int32_t shells_in_range,
                                                         int64_t nside, size_t bytes) {
    if (n < 0 || n_rep < 0 || n_rep > 64 || shells_in_range < 1 || nside < 1 || nside > UFALCON_MAX_NSIDE)
        return 0;
    const int side = 2 * n_rep + 1;
    PartLayout L;
    if (!plan_layout(L, n, (int64_t)shells_in_range * npix_of(nside), side * side * side, bytes, 0) || L.total > bytes)
        return 0;
    return (int64_t)L.budget;
}

extern "C" size_t ufalcon_bin_shells_workspace_size_partitioned(int64_t n, int32_t n_rep, int32_t shells_in_range,
                                                                int64_t nside, int64_t max_keys) {
    if (n < 0 || n_rep < 0 || n_rep > 64 || shells_in_range < 1 || nside < 1 || nside > UFALCON_MAX_NSIDE ||
        max_keys < 0)
        return 0;
    const int side = 2 * n_rep + 1;
    const int img = side * side * side;
    // the layout keeps room for the claim protocol on top of max_keys
    return partitioned_workspace_size(n, (int64_t)shells_in_range * npix_of(nside), img, max_keys > 0 ? max_keys : 1);
}
