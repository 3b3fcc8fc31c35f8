// Host-side helpers shared by the ufalcon entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdint>

#include "../../include/ufalcon.h"

namespace ufx {

#define UFX_HIP_CHECK(expr)                            \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return UFALCON_EHIP;     \
    } while (0)

inline hipStream_t as_stream(ufalcon_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// roctx range around one entry point call.
struct ApiRange {
    explicit ApiRange(const char *name) { roctxRangePushA(name); }
    ~ApiRange() { roctxRangePop(); }
    ApiRange(const ApiRange &) = delete;
    ApiRange &operator=(const ApiRange &) = delete;
};

// True when UFALCON_FAULT_INJECT names `point` (defined in bin_shells.hip).
bool fault_injected(const char *point);

// First statement of an entry point that returns a status.
#define UFX_API_ENTRY(name)                 \
    ::ufx::ApiRange ufx_api_range_(name);  \
    if (::ufx::fault_injected(name)) return UFALCON_EINJECTED
// First statement of a destroy call: traced, never failed.
#define UFX_API_RANGE(name) ::ufx::ApiRange ufx_api_range_(name)

inline int check_edges(const double *e, int32_t n_shells) {
    if (!e) return UFALCON_EINVAL;
    if (n_shells < 1) return UFALCON_EINVAL;
    if (n_shells > UFALCON_MAX_SHELLS) return UFALCON_ETOO_MANY_SHELLS;
    for (int32_t j = 0; j <= n_shells; ++j) {
        if (!std::isfinite(e[j]) || e[j] < 0.0) return UFALCON_EUNSORTED_EDGES;
        if (j > 0 && !(e[j] > e[j - 1])) return UFALCON_EUNSORTED_EDGES;
    }
    return UFALCON_OK;
}

inline int check_nside(int64_t nside) {
    return (nside >= 1 && nside <= UFALCON_MAX_NSIDE) ? UFALCON_OK : UFALCON_ENSIDE;
}

inline int64_t npix_of(int64_t nside) { return 12 * nside * nside; }

// Grid for a flat kernel over `work` items with `per_block` items per block.
inline unsigned blocks_for(int64_t work, int64_t per_block, unsigned cap = 1u << 20) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (unsigned)(b > (int64_t)cap ? cap : b);
}

// Cross-stream ordering hooks of a partitioned binning call (batched pipelines):
// the first key pass waits for `wait_keys`, and `done_keys` is recorded right
// after it, so that consecutive realisations on two streams start their key
// passes one after another and the rest of their work overlaps.  Null events
// are skipped.
struct PartHooks {
    hipEvent_t wait_keys = nullptr;
    hipEvent_t done_keys = nullptr;
};

// Record the end of a phase on the timer (no-op for a null timer).  Defined in timer.hip.
void timer_start(ufalcon_phase_timer *t, hipStream_t s);
void timer_mark(ufalcon_phase_timer *t, int phase, hipStream_t s);

// Upper bound on the number of instances a single (shell, pixel) cell can receive
// from n particles with images {-R..R}^3 of a box of side L: the cell of shell b
// has diameter <= (e_{b+1} - e_b) + e_{b+1} * psi(nside) with psi an upper bound
// on a pixel's angular diameter, and a set of diameter D holds at most
// (floor(D/L) + 1)^3 lattice translates of one point.
double cell_instance_bound(int64_t n, double L, int32_t R, const double *e, int32_t b0, int32_t b1, int64_t nside);

// Pixel angular-diameter bound used above (radians).
inline double pixel_diameter_bound(int64_t nside) {
    double psi = 4.0 / (double)nside;
    return psi > M_PI ? M_PI : psi;
}

}  // namespace ufx
