// Host build of the library's device-side decision code (exact.hpp, ring.hpp)
// so that its logic can be checked against the oracle on a machine without a GPU.
#define UFX_HOST_BUILD 1
#include "../../paper_1801_05745_amd/csrc/exact.hpp"
#include "../../paper_1801_05745_amd/csrc/ring.hpp"

extern "C" {
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
int shim_fast_shell(const double *e2, int nb, double r2, int *clear) {
    int steps = 0;
    while ((2 << steps) <= nb + 1) ++steps;
    bool c = false;
    int j = ufx::fast_shell(e2, nb, steps, r2, c);
    *clear = c ? 1 : 0;
    return j;
}
double shim_tt(double dx, double dy) {
    ufx::dd t = ufx::tt_dd(dx, dy);
    return t.hi;
}
}
