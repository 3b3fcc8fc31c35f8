// Host build of the library's device-side decision code (exact.hpp, ring.hpp)
// so that its logic can be checked against the oracle on a machine without a GPU.
#define UFX_HOST_BUILD 1
#define UFX_HOST_ESTIMATE_MODEL 1
#include <cmath>
#include <cstring>
#include <vector>

#include "../../paper_1801_05745_amd/csrc/exact.hpp"
#include "../../paper_1801_05745_amd/csrc/ring.hpp"

// Model of the device's reciprocal estimates: the IEEE value times (1 + s e),
// with e and the sign s set by the test (s = 0: a sign from the input's bits).
static double g_est_err = 0.0;
static int g_est_sign = 1;
static double perturb(double exact, double x) {
    int s = g_est_sign;
    if (s == 0) {
        uint64_t b;
        std::memcpy(&b, &x, sizeof b);
        b ^= b >> 29;
        b *= 0xBF58476D1CE4E5B9ull;
        s = ((b >> 61) & 1) ? 1 : -1;
    }
    return exact * (1.0 + s * g_est_err);
}
double ufx::host_rsq_estimate(double x) { return perturb(1.0 / std::sqrt(x), x); }
double ufx::host_rcp_estimate(double x) { return perturb(1.0 / x, x); }

extern "C" {
void shim_set_estimate_error(double err, int sign) {
    g_est_err = err;
    g_est_sign = sign;
}
int64_t shim_exact_ring_pixel(int64_t nside, double dx, double dy, double dz, int *unresolved) {
    *unresolved = 0;
    return ufx::exact_ring_pixel(nside, dx, dy, dz, unresolved);
}
int shim_exact_shell(double dx, double dy, double dz, const double *e, int nb) {
    return ufx::exact_shell(dx, dy, dz, e, nb);
}
int shim_fast_ring_pixel(int64_t nside, double dx, double dy, double dz, int64_t *pix) {
    int32_t p = -1;
    const int ok = ufx::fast_ring_pixel((int32_t)nside, (double)nside, ufx::floor_margin((double)nside), dx, dy, dz, p) ? 1 : 0;
    *pix = p;
    return ok;
}
double shim_fast_tt(double dx, double dy) { return ufx::fast_tt(dx, dy); }
// fast_shell on squared edges e2[0..nb]; use_table selects the lookup-table form
// (cells over [lo2, hi2) as the library builds them), else the binary search.
// Returns -100 when a table was asked for and the edges admit none.
int shim_fast_shell(const double *e2, int nb, double r2, int *clear, int use_table, double lo2, double hi2) {
    int steps = 0;
    while ((2 << steps) <= nb + 1) ++steps;
    std::vector<double> pad(nb + 5);
    pad[0] = pad[1] = -ufx::kEdgeSentinel;
    for (int j = 0; j <= nb; ++j) pad[j + 2] = e2[j];
    pad[nb + 3] = pad[nb + 4] = ufx::kEdgeSentinel;
    const double *E = pad.data() + 2;
    int tab_n = 0;
    double h = 0.0, scale = 0.0;
    std::vector<int16_t> tab;
    if (use_table) {
        tab_n = ufx::shell_table_cells(e2, nb, lo2, hi2);
        if (!tab_n) return -100;
        h = (hi2 - lo2) / tab_n;
        scale = tab_n / (hi2 - lo2);
        tab.resize(tab_n);
        for (int t = 0; t < tab_n; ++t)
            tab[t] = ufx::shell_table_entry(E, nb, steps, lo2 + (double)t * h,
                                            t + 1 < tab_n ? lo2 + (double)(t + 1) * h : hi2);
    }
    bool c = false;
    int j = ufx::fast_shell(E, nb, steps, tab.data(), tab_n, lo2, scale, r2, c);
    *clear = c ? 1 : 0;
    return j;
}
double shim_tt(double dx, double dy) {
    ufx::dd t = ufx::tt_dd(dx, dy);
    return t.hi;
}
}
