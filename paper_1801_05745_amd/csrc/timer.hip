// Caller-owned phase timer of the binning call: HIP events recorded on the
// call's stream at phase boundaries, read back as per-phase milliseconds.
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/ufalcon.h"
#include "internal.hpp"

struct ufalcon_phase_timer {
    hipEvent_t ev[UFALCON_TIMER_EVENTS];
    int32_t phase[UFALCON_TIMER_EVENTS];  // phase that ends at event i (-1: the start marker)
    int32_t used;
    int32_t overflow;
};

namespace ufx {

void timer_start(ufalcon_phase_timer *t, hipStream_t s) {
    if (!t) return;
    t->used = 0;
    t->overflow = 0;
    timer_mark(t, -1, s);
}

void timer_mark(ufalcon_phase_timer *t, int phase, hipStream_t s) {
    if (!t) return;
    if (t->used >= UFALCON_TIMER_EVENTS) {
        t->overflow = 1;
        return;
    }
    if (hipEventRecord(t->ev[t->used], s) != hipSuccess) {
        t->overflow = 1;
        return;
    }
    t->phase[t->used++] = phase;
}

}  // namespace ufx

extern "C" int ufalcon_phase_timer_create(ufalcon_phase_timer **timer) {
    UFX_API_ENTRY("ufalcon_phase_timer_create");
    if (!timer) return UFALCON_EINVAL;
    *timer = nullptr;
    auto *t = new (std::nothrow) ufalcon_phase_timer();
    if (!t) return UFALCON_EINVAL;
    for (int i = 0; i < UFALCON_TIMER_EVENTS; ++i) {
        if (hipEventCreate(&t->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(t->ev[j]);
            delete t;
            return UFALCON_EHIP;
        }
    }
    t->used = 0;
    t->overflow = 0;
    *timer = t;
    return UFALCON_OK;
}

extern "C" int ufalcon_phase_timer_destroy(ufalcon_phase_timer *timer) {
    UFX_API_RANGE("ufalcon_phase_timer_destroy");
    if (!timer) return UFALCON_OK;
    int rc = UFALCON_OK;
    for (int i = 0; i < UFALCON_TIMER_EVENTS; ++i)
        if (hipEventDestroy(timer->ev[i]) != hipSuccess) rc = UFALCON_EHIP;
    delete timer;
    return rc;
}

extern "C" int ufalcon_phase_timer_read(ufalcon_phase_timer *timer, double *ms) {
    UFX_API_ENTRY("ufalcon_phase_timer_read");
    if (!timer || !ms || timer->used < 1) return UFALCON_EINVAL;
    for (int k = 0; k < UFALCON_NPHASES; ++k) ms[k] = 0.0;
    if (hipEventSynchronize(timer->ev[timer->used - 1]) != hipSuccess) return UFALCON_EHIP;
    for (int i = 1; i < timer->used; ++i) {
        float dt = 0.0f;
        if (hipEventElapsedTime(&dt, timer->ev[i - 1], timer->ev[i]) != hipSuccess) return UFALCON_EHIP;
        const int ph = timer->phase[i];
        if (ph >= 0 && ph < UFALCON_NPHASES) ms[ph] += (double)dt;
    }
    return timer->overflow ? UFALCON_EOVERFLOW : UFALCON_OK;
}

extern "C" int ufalcon_phase_timer_intervals(const ufalcon_phase_timer *timer, int32_t *counts) {
    UFX_API_ENTRY("ufalcon_phase_timer_intervals");
    if (!timer || !counts || timer->used < 1) return UFALCON_EINVAL;
    for (int k = 0; k < UFALCON_NPHASES; ++k) counts[k] = 0;
    for (int i = 1; i < timer->used; ++i) {
        const int ph = timer->phase[i];
        if (ph >= 0 && ph < UFALCON_NPHASES) ++counts[ph];
    }
    return timer->overflow ? UFALCON_EOVERFLOW : UFALCON_OK;
}
