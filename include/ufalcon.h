/*
 * ufalcon — MI355X (gfx950) library for the data-parallel hot path of the
 * UFalcon multi-lens-plane method (Sgier, Refregier, Amara & Nicola,
 * "Fast Generation of Covariance Matrices for Weak Lensing", arXiv:1801.05745):
 * particles -> (radial shell, HEALPix RING pixel) count maps, then the Born
 * convergence sum kappa[p] = sum_b W_b (n_b[p]/nbar_b - 1), with its adjoint and
 * batched forms.
 *
 * Conventions for every entry point
 *   - Return value: UFALCON_OK (0) or a negative ufalcon_err code; nothing
 *     throws across this boundary.  ufalcon_strerror() names a code.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are read before the call returns and may be reused at once.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream) and is
 *     asynchronous; outputs are valid after the stream is synchronised.
 *   - Conditions found on the device (non-finite inputs, guard-band fallbacks)
 *     are added to a caller-owned device ufalcon_status.
 *   - Count maps are uint32 [n_shells][12*nside^2], row-major, and binning
 *     ADDS to them, so chunks, nested boxes and subvolumes compose; the caller
 *     zeroes them (ufalcon_fill_u32).
 *   - Arguments are validated on the host before anything is enqueued; on an
 *     error return nothing has been enqueued.
 */
#ifndef UFALCON_H
#define UFALCON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ufalcon_stream_t; /* hipStream_t */

typedef enum ufalcon_err {
    UFALCON_OK = 0,
    UFALCON_EINVAL = -1,          /* null pointer, negative size, bad enum value */
    UFALCON_EUNSORTED_EDGES = -2, /* shell edges not finite, >= 0 and strictly ascending */
    UFALCON_ENSIDE = -3,          /* nside outside [1, 8192] */
    UFALCON_EOVERFLOW = -4,       /* a uint32 count cell could exceed 2^32 - 1 */
    UFALCON_EWORKSPACE = -5,      /* workspace missing or too small */
    UFALCON_EHIP = -6,            /* a HIP runtime call failed */
    UFALCON_ETOO_MANY_SHELLS = -7, /* more than UFALCON_MAX_SHELLS shells or UFALCON_MAX_BINS source bins */
    UFALCON_EINJECTED = -8         /* failure injected by UFALCON_FAULT_INJECT (tests of error handling) */
} ufalcon_err;

/* Instrumentation of every entry point that returns a status:
 *   - a roctx range named after the entry point (rocprofv3 --marker-trace shows
 *     the library calls around their kernels);
 *   - fault injection for tests of error propagation: when the environment
 *     variable UFALCON_FAULT_INJECT holds the entry point's name (a
 *     comma-separated list; "*" names every entry point), the call returns
 *     UFALCON_EINJECTED at once, before it validates or touches any argument.
 *     The name "partition_chunk" makes the partitioned binning path fail after
 *     the kernels of its first chunk are enqueued: the call returns
 *     UFALCON_EINJECTED although work was queued and the count map was
 *     partly updated, which is what a caller must never treat as a result.
 *     The destroy calls are never failed.  The variable is read on every call. */

#define UFALCON_MAX_SHELLS 256
#define UFALCON_MAX_NSIDE 8192
#define UFALCON_MAX_BINS 8
#define UFALCON_NPARAM 4 /* derivative slots: 0 Omega_m, then the source parameters */

typedef enum ufalcon_dtype { UFALCON_F32 = 0, UFALCON_F64 = 1 } ufalcon_dtype;

/* Device-side counters, accumulated by binning calls (zero it to start). */
typedef struct ufalcon_status {
    unsigned long long n_instances;  /* particle images counted into a (shell, pixel) cell */
    unsigned long long n_invalid;    /* particles skipped for a non-finite coordinate */
    unsigned long long n_guarded;    /* instances decided by the exact path (near a boundary) */
    unsigned long long n_unresolved; /* instances the exact path could not certify (expected 0) */
    unsigned long long n_fallback;   /* instances of the partitioned path added by a global atomic because
                                        the chunk's key buffer was full (exact, but slow; expected 0) */
} ufalcon_status;

const char *ufalcon_strerror(int code);
int ufalcon_version(void);

/* Fill n uint32 words with `value` (a kernel, not a memset: safe inside graph capture). */
int ufalcon_fill_u32(uint32_t *p, int64_t n, uint32_t value, ufalcon_stream_t stream);

/*
 * Count maps as int64 (section 2.3 eq. (5): n_p counts particles; a caller
 * that keeps 64-bit maps, or adds more calls into one map than a uint32 cell
 * can hold, bins each call into uint32 and widens or accumulates here):
 *   out[i] = counts[i]            (accumulate = 0)
 *   out[i] = out[i] + counts[i]   (accumulate = 1)
 * counts device uint32[n]; out device int64[n].  Errors: EINVAL, EHIP.
 */
int ufalcon_counts_to_i64(const uint32_t *counts, int64_t n, int64_t *out, int accumulate, ufalcon_stream_t stream);

/*
 * Shell binning (section 2.3 eq. (5): n_p(pix, Delta chi_b), the number of
 * particles of shell b in pixel pix; section 2.4 eq. (8): shells by comoving
 * radius with the observer at the box centre; section 2.4: HEALPix RING
 * pixelisation with 12*nside^2 pixels, subvolume maps summed).
 *
 * x, y, z      device SoA positions, n values each, dtype UFALCON_F32 or UFALCON_F64,
 *              comoving Mpc/h; a particle with a non-finite coordinate is
 *              skipped and counted in status->n_invalid.
 * observer     host double[3].
 * box_L, n_rep periodic images s in {-n_rep..n_rep}^3 of every particle are
 *              binned: d = fl64(fl64(x - o) + fl64(s * box_L)) per axis
 *              (n_rep = 0: no replication).
 * chi_edges    host double[n_shells + 1], finite, >= 0, strictly ascending.
 * shell range  only shells b in [shell_begin, shell_end) are binned
 *              (nesting: one source per shell range).
 * counts       device uint32 [n_shells][12*nside^2]; cell (b, pix) += 1 for every
 *              instance with chi_b <= |d| < chi_{b+1} (half-open) and RING pixel pix
 *              of the direction d.
 * Exactness: every count equals the exact-real function of the FP64 d; FP64
 * decisions near a boundary are re-taken exactly on the device and counted
 * in status->n_guarded.
 * workspace    device, 256-byte aligned, at least ufalcon_bin_shells_workspace_size(0)
 *              bytes: it lists the guarded instances for the exact pass.  A larger
 *              one (ufalcon_bin_shells_workspace_size(k) lists k) avoids a second
 *              walk over all images when more than that many are guarded.  Calls
 *              sharing a workspace must be stream-ordered.
 * Accumulation: with a workspace of at least
 *              ufalcon_bin_shells_workspace_size_partitioned(n, n_rep, shell_end - shell_begin,
 *              nside, k) bytes (k = keys per chunk, e.g. n * (2 n_rep + 1)^3), the
 *              counts are accumulated by the partitioned path (keys emitted, radix-
 *              partitioned by cell block, counted in LDS; particles are processed in
 *              device-planned chunks when the keys exceed the workspace); with a
 *              smaller one, by one global atomic per instance.  Both give identical maps.
 * Errors: EINVAL, EUNSORTED_EDGES, ENSIDE, ETOO_MANY_SHELLS, EWORKSPACE, EOVERFLOW
 * (host bound on the instances one cell can receive in this call exceeds
 * 2^32 - 1), EHIP.
 */
size_t ufalcon_bin_shells_workspace_size(int64_t max_listed);
size_t ufalcon_bin_shells_workspace_size_partitioned(int64_t n, int32_t n_rep, int32_t shells_in_range,
                                                     int64_t nside, int64_t max_keys);
/* Keys one chunk of the partitioned accumulation takes at least with a workspace
 * of `bytes` (host computation, no device call; the layout assumes all
 * (2 n_rep + 1)^3 images can reach the range); 0 when that workspace selects
 * the atomic path or an argument is out of range.  A workspace of
 * ufalcon_bin_shells_workspace_size_partitioned(..., k) bytes holds at least k. */
int64_t ufalcon_bin_shells_partition_capacity(int64_t n, int32_t n_rep, int32_t shells_in_range, int64_t nside,
                                              size_t bytes);
int ufalcon_bin_shells(const void *x, const void *y, const void *z, int64_t n, int dtype,
                       const double *observer, double box_L, int32_t n_rep,
                       const double *chi_edges, int32_t n_shells, int32_t shell_begin, int32_t shell_end,
                       int64_t nside, uint32_t *counts, ufalcon_status *status,
                       void *workspace, size_t workspace_bytes, ufalcon_stream_t stream);

/*
 * Binning without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as ufalcon_bin_shells minus
 * the workspace; counts are accumulated by one global atomic per instance (the
 * path ufalcon_bin_shells takes with a small workspace).  Its scratch memory
 * (a 256-byte guard-list header and up to UFALCON_NOALLOC_GUARD_ENTRIES listed
 * guarded instances of 32 bytes: 2 MiB + 256 bytes) is a
 * file-scope device array that every GPU the library runs on holds until the
 * process ends; no input size needs more (instances beyond the list's capacity
 * are decided by the rescue pass).  The first call on a device looks the array
 * up (hipGetSymbolAddress); no call allocates or frees memory.  All calls on
 * one GPU share that GPU's array: calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and must be serialised
 * by the caller.  Errors: those of ufalcon_bin_shells except EWORKSPACE; EHIP
 * also when the array's address cannot be obtained.
 */
#define UFALCON_NOALLOC_GUARD_ENTRIES 65536
int ufalcon_bin_shells_noalloc(const void *x, const void *y, const void *z, int64_t n, int dtype,
                               const double *observer, double box_L, int32_t n_rep,
                               const double *chi_edges, int32_t n_shells, int32_t shell_begin, int32_t shell_end,
                               int64_t nside, uint32_t *counts, ufalcon_status *status, ufalcon_stream_t stream);

/*
 * Phase timing of a binning call (diagnostics: results do not depend on it).
 * A timer owns HIP events created on the device current at
 * ufalcon_phase_timer_create.  ufalcon_bin_shells_timed takes the same
 * arguments as ufalcon_bin_shells plus a timer, and records the timer's events
 * on `stream` between the phases of the call:
 *   SETUP       guard-list reset and chunk plan
 *   DECIDE      shell and RING-pixel decisions of every image (the key pass of
 *               partitioned accumulation, or the atomic pass)
 *   PARTITION   the two radix partition levels of the keys
 *   ACCUMULATE  per-cell-block LDS histograms added into `counts`
 *   EXACT       exact decisions of guarded instances (and the rescue pass)
 * ufalcon_phase_timer_read waits for the last recorded event and writes the
 * milliseconds of each phase, summed over chunks, to ms[UFALCON_NPHASES].
 * ufalcon_phase_timer_intervals writes how many intervals each phase's sum
 * covers to counts[UFALCON_NPHASES] (DECIDE: one per key-pass launch, i.e. per
 * chunk of a partitioned call), without waiting.
 * A timer serves one call at a time; each timed call replaces the previous
 * record.  Errors: EINVAL (null timer / ms / counts, or read before any timed
 * call), EOVERFLOW (more than UFALCON_TIMER_EVENTS events were needed: the
 * record is incomplete), EHIP.
 */
#define UFALCON_TIMER_EVENTS 256
enum {
    UFALCON_PHASE_SETUP = 0,
    UFALCON_PHASE_DECIDE = 1,
    UFALCON_PHASE_PARTITION = 2,
    UFALCON_PHASE_ACCUMULATE = 3,
    UFALCON_PHASE_EXACT = 4,
    UFALCON_NPHASES = 5
};
typedef struct ufalcon_phase_timer ufalcon_phase_timer;
int ufalcon_phase_timer_create(ufalcon_phase_timer **timer);
int ufalcon_phase_timer_destroy(ufalcon_phase_timer *timer);
int ufalcon_bin_shells_timed(const void *x, const void *y, const void *z, int64_t n, int dtype,
                             const double *observer, double box_L, int32_t n_rep,
                             const double *chi_edges, int32_t n_shells, int32_t shell_begin, int32_t shell_end,
                             int64_t nside, uint32_t *counts, ufalcon_status *status,
                             void *workspace, size_t workspace_bytes, ufalcon_stream_t stream,
                             ufalcon_phase_timer *timer);
int ufalcon_phase_timer_read(ufalcon_phase_timer *timer, double *ms);
int ufalcon_phase_timer_intervals(const ufalcon_phase_timer *timer, int32_t *counts);

/* Source redshift distributions for the lensing weights. */
typedef enum ufalcon_source_kind { UFALCON_SOURCE_DELTA = 0, UFALCON_SOURCE_SMAIL = 1 } ufalcon_source_kind;

typedef struct ufalcon_source {
    int32_t kind;  /* ufalcon_source_kind */
    double z_s;    /* DELTA: source redshift (derivative slot 1) */
    double alpha;  /* SMAIL n(z) ~ z^alpha exp(-(z/z0)^beta) on [0, z_max]: slot 1 */
    double beta;   /* slot 2 */
    double z0;     /* slot 3 */
    double z_max;  /* support end (not differentiated) */
} ufalcon_source;

/*
 * Comoving distance chi(z) = (c/H0) int_0^z dz'/E(z') in Mpc/h for flat
 * LambdaCDM, E = sqrt(Om (1+z)^3 + 1 - Om) (section 2.3: D(z) = (H0/c) chi(z)).
 * z, chi: device double[n].
 */
int ufalcon_comoving_distance(const double *z, int64_t n, double omega_m, double *chi, ufalcon_stream_t stream);

/*
 * Born lensing weights of each shell for T source bins (section 2.3 eqs. (1)-(3),
 * (6)): W[t][b] = (3/2) Om int over the shell of (1+z) D(z) q_t(z) dD, with
 * q = 1 - D/D_s for a delta source (zero behind it) and
 * q = int_z^{z_max} nhat(z') (1 - D(z)/D(z')) dz' for an n(z).  The comoving
 * edges stay fixed when Omega_m changes (their redshifts move).
 * chi_edges host double[n_shells+1]; sources host [T]; W device double[T][n_shells];
 * dW device double[T][n_shells][UFALCON_NPARAM] (dW/dOmega_m and dW/d source
 * parameters, forward-mode) or NULL.
 */
int ufalcon_lensing_weights(double omega_m, const ufalcon_source *sources, int32_t T,
                            const double *chi_edges, int32_t n_shells, double *W, double *dW,
                            ufalcon_stream_t stream);

/* grad_theta[t][k] = sum_b grad_W[t][b] * dW[t][b][k] (device, double). */
int ufalcon_lensing_weights_vjp(const double *dW, const double *grad_W, int32_t T, int32_t n_shells,
                                double *grad_theta, ufalcon_stream_t stream);

typedef enum ufalcon_nbar_mode { UFALCON_NBAR_EXACT_VOLUME = 0, UFALCON_NBAR_LOWER_EDGE = 1 } ufalcon_nbar_mode;

/*
 * 1/nbar_b for shells [shell_begin, shell_end): nbar_b = (n_src / box_L^3) V_b / N_pix
 * with V_b = (4 pi/3)(chi_{b+1}^3 - chi_b^3) (EXACT_VOLUME) or 4 pi chi_b^2 Delta chi_b
 * (LOWER_EDGE, eq. (6) literally); section 2.3 eq. (5): rho ~ m_p N / V.
 * inv_nbar: device double[n_shells]; entries outside the range are not written.
 */
int ufalcon_inv_nbar(int64_t n_src, double box_L, const double *chi_edges, int32_t n_shells,
                     int32_t shell_begin, int32_t shell_end, int64_t nside, int32_t mode,
                     double *inv_nbar, ufalcon_stream_t stream);

/*
 * Born convergence (section 2.3 eq. (6)):
 *   kappa[t][p] = sum_b W[t][b] * (counts[b][p] * inv_nbar[b] - 1)
 * accumulated in FP64 in shell order, rounded once to out_dtype.
 * counts device uint32 [n_shells][npix]; W device double[T][n_shells];
 * inv_nbar device double[n_shells]; kappa device [T][npix] of out_dtype.
 */
int ufalcon_born_kappa(const uint32_t *counts, int32_t n_shells, int64_t nside, const double *W,
                       const double *inv_nbar, int32_t T, void *kappa, int out_dtype, ufalcon_stream_t stream);

/*
 * Projected overdensity (section 2.3 eq. (7)): the Born sum with weights
 * Delta chi_b / sum_b Delta chi_b over shells [0, n_shells).  delta device [npix].
 */
int ufalcon_overdensity(const uint32_t *counts, int32_t n_shells, int64_t nside, const double *chi_edges,
                        const double *inv_nbar, void *delta, int out_dtype, ufalcon_stream_t stream);

/*
 * Adjoint of the Born sum with respect to the weights:
 *   grad_W[t][b] = sum_p grad_kappa[t][p] * (counts[b][p] * inv_nbar[b] - 1)
 * as a deterministic two-stage FP64 reduction (fixed order, bitwise
 * reproducible).  grad_kappa device [T][npix] of grad_dtype; grad_W device
 * double[T][n_shells]; workspace device, at least
 * ufalcon_born_kappa_adjoint_workspace_size() bytes.
 */
size_t ufalcon_born_kappa_adjoint_workspace_size(int32_t n_shells, int64_t nside, int32_t T);
int ufalcon_born_kappa_adjoint(const uint32_t *counts, int32_t n_shells, int64_t nside, const double *inv_nbar,
                               const void *grad_kappa, int grad_dtype, int32_t T, double *grad_W,
                               void *workspace, size_t workspace_bytes, ufalcon_stream_t stream);

/*
 * Batched form: many realisations (section 2.2 and 3.2: 150 independent maps
 * for the covariance) with uneven particle counts and shell sets, binned by
 * one persistent launch over a work queue of (realisation, tile) items and
 * reduced by one batched Born launch.  A plan holds device copies of the
 * descriptors and may hold a captured HIP graph.
 */
typedef struct ufalcon_batch_item {
    const void *x, *y, *z;     /* device positions */
    int64_t n;                 /* particles */
    double observer[3];
    double box_L;
    int32_t n_rep;
    int32_t n_shells;          /* shells of this realisation */
    int32_t shell_begin, shell_end;
    const double *chi_edges;   /* host double[n_shells+1] (copied into the plan) */
    uint32_t *counts;          /* device [n_shells][npix] */
    const double *W;           /* device double[T][n_shells] (for the Born launch) */
    const double *inv_nbar;    /* device double[n_shells] */
    void *kappa;               /* device [T][npix] of the plan's out_dtype */
} ufalcon_batch_item;

typedef struct ufalcon_batch_plan ufalcon_batch_plan;

typedef enum ufalcon_accumulation {
    UFALCON_ACCUMULATE_PARTITIONED = 0, /* keys + radix partition + LDS block histograms, realisations on two
                                           streams with their key passes staggered */
    UFALCON_ACCUMULATE_ATOMIC = 1,      /* one persistent launch over (realisation, tile), global atomics with
                                           equal keys aggregated across each wavefront */
    UFALCON_ACCUMULATE_AUTO = 2,        /* the autotuner's choice for this batch shape (else PARTITIONED) */
    UFALCON_ACCUMULATE_PARTITIONED_ONE_STREAM = 3 /* partitioned, realisations one after another */
} ufalcon_accumulation;

/*
 * Realisations may share a count map: snapshots bound to disjoint shell ranges of
 * one map (section 2.4's nested boxes), or subvolumes binned into the same shells
 * (counts add).  Realisations whose written rows overlap are binned one after
 * another; the Born launch of such a plan computes each realisation's kappa from
 * its whole map (use T = 0 and one ufalcon_born_kappa call on the shared map).
 *
 * tile: particles per work item of the persistent kernel (0 = default, or the
 * autotuner's choice under UFALCON_ACCUMULATE_AUTO); persistent_wgs: its
 * workgroups (0 likewise); accumulation: ufalcon_accumulation.
 * The partitioned form allocates one device workspace for the largest realisation
 * at plan creation (never on the binning calls).
 */
int ufalcon_batch_plan_create(const ufalcon_batch_item *items, int32_t n_items, int dtype, int64_t nside,
                              int32_t T, int out_dtype, int64_t tile, int32_t persistent_wgs,
                              int32_t accumulation, ufalcon_batch_plan **plan);
int ufalcon_batch_plan_destroy(ufalcon_batch_plan *plan);
/* Zero every count map of the plan. */
int ufalcon_batch_clear(ufalcon_batch_plan *plan, ufalcon_stream_t stream);
int ufalcon_bin_shells_batched(ufalcon_batch_plan *plan, ufalcon_status *status, ufalcon_stream_t stream);
int ufalcon_born_kappa_batched(ufalcon_batch_plan *plan, ufalcon_stream_t stream);
/* clear + bin + Born for the whole batch as one captured HIP graph (captured on first use, replayed after). */
int ufalcon_batch_run_graph(ufalcon_batch_plan *plan, ufalcon_status *status, ufalcon_stream_t stream);

/*
 * Autotuner of the batched form.  Times clear + bin + Born of the first
 * min(n_items, sample_items) realisations (sample_items <= 0: all) under each
 * candidate configuration: partitioned accumulation on two streams and on one,
 * and the persistent atomic kernel (aggregated equal keys) with 2^18-particle
 * tiles and 8 workgroups per compute unit, and 2^16-particle tiles and 16.
 * Each candidate runs once to warm up and three times timed (HIP events on
 * `stream`; the call synchronises); its median is its time.  The fastest is
 * written to *tuning and recorded in a process-wide cache keyed by the batch
 * shape (GPU architecture and compute units, dtype, nside, T, number of
 * realisations, log2 of the particle total, largest n_rep);
 * ufalcon_batch_plan_create with UFALCON_ACCUMULATE_AUTO, tile 0 and
 * persistent_wgs 0 takes the cached choice.  The cache is the library's only
 * global state (mutex-guarded); ufalcon_batch_tuning_save and _load persist it.
 * Side effects: the sampled realisations' counts and kappa are overwritten;
 * plans are created and freed (device allocations happen here, never in the
 * binning calls of a plan).
 */
#define UFALCON_TUNE_MAX 16
typedef struct ufalcon_batch_tuning {
    int32_t accumulation;     /* chosen ufalcon_accumulation (PARTITIONED or ATOMIC) */
    int32_t persistent_wgs;   /* chosen workgroups (ATOMIC) */
    int64_t tile;             /* chosen particles per work item (ATOMIC) */
    int32_t n_tried;          /* candidates timed */
    int32_t best;             /* index of the chosen candidate */
    double ms[UFALCON_TUNE_MAX];            /* time of each candidate, in the order listed above */
    int32_t cand_accumulation[UFALCON_TUNE_MAX];
    int32_t cand_wgs[UFALCON_TUNE_MAX];
    int64_t cand_tile[UFALCON_TUNE_MAX];
} ufalcon_batch_tuning;
int ufalcon_batch_autotune(const ufalcon_batch_item *items, int32_t n_items, int dtype, int64_t nside, int32_t T,
                           int out_dtype, int32_t sample_items, ufalcon_batch_tuning *tuning,
                           ufalcon_stream_t stream);

/*
 * Persisted tuning choices: _save writes every cached choice to the file at
 * `path` (one JSON object per line: arch, cus, dtype, nside, T, items, log2n,
 * max_rep, accumulation, wgs, tile); _load adds the choices of such a file to
 * the cache (entries already cached are replaced) and writes how many it read
 * to *n_loaded (may be NULL).  Host only.  Errors: EINVAL (null path, or a line
 * that is not such an object), EHIP (the file cannot be opened or written).
 */
int ufalcon_batch_tuning_save(const char *path);
int ufalcon_batch_tuning_load(const char *path, int32_t *n_loaded);

/*
 * Spherical-harmonic coefficients of HEALPix RING maps (section 3.1: the
 * harmonic analysis behind the power spectrum of eq. (9), done there with
 * ANAFAST up to lmax = 3 Nside - 1).  The pixel quadrature
 *   a_lm = (4 pi / N_pix) sum_p map_p conj(Y_lm(theta_p, phi_p)),  0 <= m <= l <= lmax,
 * at the pixel centres, Y_lm with the Condon-Shortley phase, evaluated in
 * FP64 with a fixed reduction order (bitwise reproducible).
 * maps device [n_maps][12 Nside^2] of dtype (UFALCON_F32 | UFALCON_F64);
 * alm device double [n_maps][n_alm][2] (re, im), n_alm = (lmax+1)(lmax+2)/2,
 * m-major: index m (2 lmax + 1 - m) / 2 + l.  Any lmax in [0, 4 * 8192] is
 * accepted (beyond 3 Nside - 1 the quadrature aliases, as ANAFAST's does).
 * workspace device, at least ufalcon_map2alm_workspace_size(nside, lmax)
 * bytes (0 for invalid arguments): ring sums, lambda_mm seeds and recurrence
 * coefficients, about 16 (lmax+1)(4 Nside) + 12 (lmax+1)(2 Nside) + 16 n_alm
 * bytes (~350 MB at Nside 1024, lmax 3071).  Returns UFALCON_EINVAL for bad
 * arguments, UFALCON_ENSIDE, UFALCON_EWORKSPACE if the workspace is short.
 */
size_t ufalcon_map2alm_workspace_size(int64_t nside, int32_t lmax);
int ufalcon_map2alm(const void *maps, int dtype, int32_t n_maps, int64_t nside, int32_t lmax, double *alm,
                    void *workspace, size_t workspace_bytes, ufalcon_stream_t stream);

/*
 * Angular power spectrum from the coefficients of a real map (section 3.1
 * eq. (9), the average over m standing for the ensemble average):
 *   C_l = (|a_l0|^2 + 2 sum_{m=1}^{l} |a_lm|^2) / (2l + 1).
 * alm device as written by ufalcon_map2alm; cl device double [n_maps][lmax+1].
 */
int ufalcon_alm2cl(const double *alm, int32_t n_maps, int32_t lmax, double *cl, ufalcon_stream_t stream);

/*
 * Covariance and correlation of power spectra over realisations (section 3.2
 * eqs. (10) and (11)).  Band b averages C_l over l in
 * [ell_min + b delta_ell, ell_min + (b+1) delta_ell) (the paper bins by
 * delta_ell = 4, 10, 24); then
 *   band_mean[b] = (1/R) sum_r X[r][b]
 *   cov[b][c]    = sum_r (X[r][b] - band_mean[b]) (X[r][c] - band_mean[c]) / (R - ddof)
 *   corr[b][c]   = cov[b][c] / (sqrt(cov[b][b]) sqrt(cov[c][c]))   (NaN where a variance is 0)
 * (eq. (10) as printed multiplies two averages; the product is averaged here).
 * cl device double [n_real][n_ell]; band_mean device [n_bands]; cov, corr
 * device [n_bands][n_bands] (corr may be NULL); ddof 0 or 1, n_real > ddof;
 * ell_min + n_bands * delta_ell <= n_ell; n_bands <= 65535.  workspace device,
 * at least ufalcon_cl_covariance_workspace_size() bytes (the band powers and
 * the standard deviations sqrt(cov[b][b])).
 */
size_t ufalcon_cl_covariance_workspace_size(int32_t n_real, int32_t n_bands);
int ufalcon_cl_covariance(const double *cl, int32_t n_real, int32_t n_ell, int32_t ell_min, int32_t delta_ell,
                          int32_t n_bands, int32_t ddof, double *band_mean, double *cov, double *corr,
                          void *workspace, size_t workspace_bytes, ufalcon_stream_t stream);

/*
 * Synthesis: the real maps whose coefficients are alm (section 3.3 smooths
 * the kappa and delta maps with a Gaussian beam before taking their PDF and
 * moments), optionally multiplied by a beam b_l:
 *   map_p = sum_l b_l [a_l0 Y_l0(p) + 2 Re sum_{m>=1} a_lm Y_lm(p)]
 * at the pixel centres (a_{l,-m} = (-1)^m conj(a_lm); Im a_l0 is ignored).
 * alm device double [n_maps][n_alm][2] (the layout of ufalcon_map2alm);
 * beam device double [lmax+1] or NULL (b_l = 1); maps device
 * [n_maps][12 Nside^2] of dtype, overwritten.  workspace device, at least
 * ufalcon_alm2map_workspace_size(nside, lmax) bytes (0 for invalid
 * arguments).  FP64 throughout, bitwise reproducible.
 */
size_t ufalcon_alm2map_workspace_size(int64_t nside, int32_t lmax);
int ufalcon_alm2map(const double *alm, int32_t n_maps, int64_t nside, int32_t lmax, const double *beam, void *maps,
                    int dtype, void *workspace, size_t workspace_bytes, ufalcon_stream_t stream);

/*
 * Gaussian beam of r.m.s. radius sigma (radians; section 3.3 uses 10.8
 * arcmin): beam[l] = exp(-l (l+1) sigma^2 / 2), l = 0..lmax, device double.
 */
int ufalcon_gaussian_beam(double sigma, int32_t lmax, double *beam, ufalcon_stream_t stream);

/*
 * One-point moments of maps of npix values (section 3.3 eqs. (12), (13)),
 * per map, in FP64 with a fixed reduction order (two passes: the mean, then
 * the central sums):
 *   [0] mean qbar      [1] m2 = (1/N) sum (q - qbar)^2     [2] m4 = (1/N) sum (q - qbar)^4
 *   [3] s^2 = m2 (eq. (12); the printed formula lacks the square)
 *   [4] sigma_{s^2}^2 = (N-1)^2/N^3 m4 - (N-1)(N-3)/N^3 m2^2   (eq. (13), mu_k -> m_k)
 * maps device [n_maps][npix] of dtype; moments device double
 * [n_maps][UFALCON_NMOMENTS]; workspace device, at least
 * ufalcon_map_moments_workspace_size(n_maps) bytes; n_maps <= 65535.
 */
#define UFALCON_NMOMENTS 5
size_t ufalcon_map_moments_workspace_size(int32_t n_maps);
int ufalcon_map_moments(const void *maps, int dtype, int32_t n_maps, int64_t npix, double *moments, void *workspace,
                        size_t workspace_bytes, ufalcon_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* UFALCON_H */
