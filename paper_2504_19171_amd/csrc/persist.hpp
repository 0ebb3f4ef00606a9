// Device-side task scheduling for persistent kernels.
//
// A persistent kernel is launched with a fixed number of workgroups; each one
// repeatedly takes the next ticket from a global counter and runs the task
// with that number.  Tickets follow a topological order of the task graph
// (every task depends only on tasks with smaller tickets), so a task that
// waits is always waiting for work that a running workgroup already owns:
// the scheme cannot deadlock, whether or not all workgroups are resident.
//
// Dependencies are counters in device memory: a producer adds 1 once its
// output is written; a consumer spins until the counter reaches the number of
// producers it needs.  Every wait is bounded by a wall-clock limit; on expiry
// the kernel records STILES_ETIMEOUT in the shared error word and every
// workgroup leaves.
//
// Coherence without cache-wide fences.  On gfx950 an agent-scope release is a
// write-back of the whole L2 of the XCD and an agent-scope acquire an
// invalidation of it; with hundreds of workgroups doing one per task these
// serialize (measured: ~15-35 us per release, and L2 re-reads falling from
// TB/s to tens of GB/s).  So data handed between workgroups of one
// persistent kernel never goes through the non-coherent caches instead: it is
// stored with device-coherent (agent-scope relaxed atomic, "sc1") stores and
// read with device-coherent loads (ld_coh / st_coh below).  A producer waits
// for its stores to complete (s_waitcnt) in every wavefront, meets the other
// wavefronts at a barrier, and only then bumps the counter; a consumer reads
// the counter with a device-coherent load and meets its wavefronts at a
// barrier before any of them loads the data.  Data written by earlier kernels
// on the stream is read with ordinary loads.
#pragma once
#include "common.hpp"
#include "../../include/stiles.h"

struct Sched {
    int* ticket;      // next ticket
    int* err;         // 0, or an error code (all workgroups stop)
    int64_t spin_limit;   // wall_clock64() ticks a wait may last
    int withhold;     // ticket whose completion is never signalled (-1: none); test hook
};

// Thread 0 takes a ticket; broadcast to the workgroup.  Returns -1 when the
// kernel is done or stopped.
__device__ inline int sched_next(const Sched& s, int ntasks, int* sh) {
    __syncthreads();
    if (threadIdx.x == 0) {
        // both requests in flight at once: a ticket taken after an error is
        // simply dropped
        const int e = ld_coh_i(s.err);
        int t = add_coh_i(s.ticket, 1);
        if (e != 0 || t >= ntasks) t = -1;
        *sh = t;
    }
    __syncthreads();
    // uniform across the workgroup: keep it (and all that derives from it) in
    // scalar registers
    return __builtin_amdgcn_readfirstlane(*sh);
}

// Wait until *flag >= target (thread 0 polls), then acquire for every thread.
// Returns false if the kernel must stop (timeout or an error elsewhere).
__device__ inline bool sched_wait(const Sched& s, int* flag, int target, int* sh) {
    if (threadIdx.x == 0) {
        int ok = 1;
        if (ld_coh_i(flag) < target) {
            const int64_t t0 = wall_clock64();
            while (ld_coh_i(flag) < target) {
                if (ld_coh_i(s.err) != 0) { ok = 0; break; }
                if (wall_clock64() - t0 > s.spin_limit) {
                    set_error_once(s.err, STILES_ETIMEOUT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        *sh = ok;
    }
    __syncthreads();
    const bool ok = __builtin_amdgcn_readfirstlane(*sh) != 0;
    __syncthreads();   // every thread has read *sh before it can be reused
    return ok;
}

// Wait until flag[i] >= target[i] for every i < n (n <= SCHED_MAX_DEPS), then
// acquire for every thread.  Thread 0 reads all the counters at once; while
// some are short it polls only the first of those (one hot counter per
// waiting workgroup: the polls of hundreds of waiting workgroups share the
// memory channels of a few counters).  Returns false if the kernel must stop.
#define SCHED_MAX_DEPS 3
// (three named slots rather than an array: an array indexed by the running
// count would live in scratch memory, whose loads count on the same memory
// counter as the task's own loads)
struct SchedDeps {
    int* f0;
    int* f1;
    int* f2;
    int t0, t1, t2;
    int n;
};
__device__ inline void deps_add(SchedDeps& d, int* flag, int target) {
    if (d.n == 0) { d.f0 = flag; d.t0 = target; }
    else if (d.n == 1) { d.f1 = flag; d.t1 = target; }
    else { d.f2 = flag; d.t2 = target; }
    ++d.n;
}
__device__ inline bool sched_wait_deps_one(const Sched& s, const int* f, int target, int64_t& t0, unsigned& polls,
                                           int x) {
    while (x < target) {
        if (t0 < 0) t0 = wall_clock64();
        // the error word is one address for every workgroup: read it on every
        // 16th poll only
        if ((polls++ & 15) == 0 && ld_coh_i(s.err) != 0) return false;
        if (wall_clock64() - t0 > s.spin_limit) {
            set_error_once(s.err, STILES_ETIMEOUT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
        x = ld_coh_i(f);
    }
    return true;
}
__device__ inline bool sched_wait_deps(const Sched& s, const SchedDeps& d, int* sh) {
    if (threadIdx.x == 0) {
        int v0 = 0, v1 = 0, v2 = 0;
        if (d.n > 0) v0 = ld_coh_i(d.f0);
        if (d.n > 1) v1 = ld_coh_i(d.f1);
        if (d.n > 2) v2 = ld_coh_i(d.f2);
        int64_t t0 = -1;
        unsigned polls = 0;
        bool ok = true;
        if (d.n > 0) ok = sched_wait_deps_one(s, d.f0, d.t0, t0, polls, v0);
        if (ok && d.n > 1) ok = sched_wait_deps_one(s, d.f1, d.t1, t0, polls, v1);
        if (ok && d.n > 2) ok = sched_wait_deps_one(s, d.f2, d.t2, t0, polls, v2);
        *sh = ok ? 1 : 0;
    }
    __syncthreads();
    const bool ok = __builtin_amdgcn_readfirstlane(*sh) != 0;
    __syncthreads();   // every thread has read *sh before it can be reused
    return ok;
}

// Add 1 to *flag once every store of this workgroup (device-coherent) has
// completed.
__device__ inline void sched_signal(const Sched& s, int* flag, int ticket) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && ticket != s.withhold) add_coh_i(flag, 1);
}

// Optional task tracing, compiled in with -DSTILES_TASK_TRACE (diagnostics
// builds only): per task, wall-clock ticks at dequeue, after its waits and
// after its signal, plus its kind / tile column / workgroup.
#ifdef STILES_TASK_TRACE
#define STILES_TRACE_MAX (1 << 20)
#define STILES_TRACE_SLOTS 8
__device__ unsigned long long g_trace[STILES_TRACE_SLOTS * STILES_TRACE_MAX];
__device__ inline void trace_rec(int t, int slot, unsigned long long v) {
    if (threadIdx.x == 0 && t >= 0 && t < STILES_TRACE_MAX) g_trace[STILES_TRACE_SLOTS * t + slot] = v;
}
#define TRACE(t, slot, v) trace_rec((t), (slot), (unsigned long long)(v))
#else
#define TRACE(t, slot, v) ((void)0)
#endif
