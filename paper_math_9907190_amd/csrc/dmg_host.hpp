// Host-side helpers shared by the 2D and 3D plans of libdmg: device guard,
// HIP-event timing of one kernel family, error mapping.
#pragma once
#include "../../include/dmg.h"
#include "dmg_common.hpp"

#include <chrono>

namespace dmg {

constexpr int kTimedMax = 64;

// Host side of a solve loop: wait until the finalize kernel has written
// evaluation it (its count of evaluations done exceeds it) or a stop into the
// pinned state h, by polling it -- no event between iterations, whose
// system-scope release would stall the queue every cycle.  Should nothing
// show within 50 ms, a stream synchronisation settles it.  The caller
// zeroes h->k and h->done before it queues the solve's first kernel.
inline int wait_evaluation(const volatile HostState* h, int it, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0; h->k < it + 1 && !h->done; spin++) {
        if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50))
            return hipStreamSynchronize(s) == hipSuccess ? MG_OK : MG_ERR_HIP;
    }
    return MG_OK;
}

// Timing of one kernel family (mg_timing_enable / mg_timing_read): every
// launch of that family is bracketed by two events on the plan's stream.
struct Timing {
    int fam = -1;
    int pend = 0;
    bool ev = false;
    hipEvent_t beg[kTimedMax], end[kTimedMax];
    double ms = 0, bytes = 0;
    long long count = 0;
    hipStream_t stream = nullptr;

    void flush()
    {
        for (int i = 0; i < pend; i++) {
            float t = 0;
            if (hipEventSynchronize(end[i]) == hipSuccess && hipEventElapsedTime(&t, beg[i], end[i]) == hipSuccess)
                ms += t;
        }
        pend = 0;
    }
    int enable(int family)
    {
        if (family >= 0 && !ev) {
            for (int i = 0; i < kTimedMax; i++)
                if (hipEventCreate(&beg[i]) != hipSuccess || hipEventCreate(&end[i]) != hipSuccess) return MG_ERR_HIP;
            ev = true;
        }
        if (ev) flush();
        fam = family;
        ms = bytes = 0;
        count = 0;
        return MG_OK;
    }
    void read(double* oms, long long* ocount, double* obytes)
    {
        if (ev) flush();
        if (oms) *oms = ms;
        if (ocount) *ocount = count;
        if (obytes) *obytes = bytes;
        ms = bytes = 0;
        count = 0;
    }
    void destroy()
    {
        if (!ev) return;
        flush();
        for (int i = 0; i < kTimedMax; i++) {
            (void)hipEventDestroy(beg[i]);
            (void)hipEventDestroy(end[i]);
        }
        ev = false;
    }
};

// Brackets one launch with events when its family is the measured one.
// The start and stop events of an open Timed bracket whose launcher times
// its single kernel itself (the dispatch records them: hipExtLaunchKernel),
// so that the figure is the kernel's own duration without the event packets
// around it.  Set only while such a bracket is open.
struct TimedSlot {
    hipEvent_t beg, end;
};
inline TimedSlot*& timed_slot()
{
    static thread_local TimedSlot* s = nullptr;
    return s;
}

// ext: the launcher in the bracket takes the events from timed_slot()
struct Timed {
    Timing* T;
    bool on, ext;
    TimedSlot slot;
    Timed(Timing* t, int fam, double bytes, bool ext_ = false) : T(t), on(t->ev && t->fam == fam), ext(ext_)
    {
        if (!on) return;
        if (T->pend == kTimedMax) T->flush();
        if (ext) {
            slot = TimedSlot{T->beg[T->pend], T->end[T->pend]};
            timed_slot() = &slot;
        } else {
            (void)hipEventRecord(T->beg[T->pend], T->stream);
        }
        T->bytes += bytes;
        T->count++;
    }
    ~Timed()
    {
        if (!on) return;
        if (ext && timed_slot() == &slot) {   // nothing took the events: an empty bracket
            (void)hipEventRecord(T->beg[T->pend], T->stream);
            (void)hipEventRecord(T->end[T->pend], T->stream);
            timed_slot() = nullptr;
        } else if (!ext) {
            (void)hipEventRecord(T->end[T->pend], T->stream);
        }
        T->pend++;
    }
};

struct DevGuard {
    int old = -1;
    bool ok = true;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) { ok = false; return; }
        if (old != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DevGuard()
    {
        if (old >= 0) {
            int cur;
            if (hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
        }
    }
};

inline int hip_status(hipError_t e) { return e == hipSuccess ? MG_OK : MG_ERR_HIP; }
inline int last_launch() { return hip_status(hipGetLastError()); }

inline int ilog2(int n)
{
    if (n < 2) return -1;
    int k = 0;
    while ((1 << k) < n) k++;
    return ((1 << k) == n) ? k : -1;
}

}  // namespace dmg
