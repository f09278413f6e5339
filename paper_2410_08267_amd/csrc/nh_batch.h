// Many requests in one persistent launch: the request descriptors, the
// per-workgroup two-slot table cache and the wave-level scheduler shared by
// the FP64 and FP32-compensated slice kernels.
//
// Each workgroup holds the coefficient tables of one or two requests in LDS
// (SLOTS).  Lanes draw trajectories from the request of the "current" slot
// through a per-request queue counter in HBM (one atomic per wavefront pass
// that has free lanes).  When that request has no unclaimed trajectories left,
// the wave holding the workgroup's lock picks another request and loads its
// table into the next slot once the lanes still running trajectories from that
// slot have finished.  With two slots the other lanes keep integrating the
// current request meanwhile; with one slot (room for a finer table) the
// workgroup drains first.  The
// integration of one trajectory is the same code as in the plain kernels and
// depends only on its own request, so results do not depend on which requests
// share a launch.
//
// A launch can also be a time slice: after a wall-clock budget the lanes stop
// claiming, store their in-flight state to HBM and the workgroup records its
// slots; the next launch restores both and continues bit for bit.  New
// requests enter between slices (continuous batching).
#pragma once

#include "nh_dp5.h"

namespace nh {

// Workgroup scheduling state in LDS.  slot_req, cur, dry and done change only
// under `lock`; active[] counts the lanes running a trajectory of each slot.
struct WgSched {
    int slot_req[2];
    int active[2];
    int cur;
    int dry;                  // the current slot's request has no unclaimed trajectories
    int lock;
    int done;                 // no request of this launch has unclaimed trajectories
};

__device__ __forceinline__ long long remaining_of(const SliceArgs &A, int r)
{
    const BatchReq &q = A.reqs[r];
    if (q.retired) return 0;
    const unsigned long long n = __hip_atomic_load(&A.next[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return n >= (unsigned long long)q.P.n_traj ? 0 : q.P.n_traj - (long long)n;
}

// Wave-cooperative choice of the next request for a workgroup; -1 if none has work.
__device__ __forceinline__ int pick_request(const SliceArgs &A)
{
    const int lane = __lane_id();
    if (A.policy == POLICY_OPEN_FIRST) {
        for (;;) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(A.cursor, 1ull);
            c = __shfl(c, 0);
            if (c >= (unsigned long long)A.n_order) break;
            const int r = A.order[c];
            if (remaining_of(A, r) > 0) return r;
        }
    } else if (A.policy == POLICY_SHARE) {
        for (int b = 0; b < A.n_order; b += 64) {
            const int i = b + lane;
            bool ok = false;
            if (i < A.n_order) {
                const int r = A.order[i];
                const long long rem = remaining_of(A, r);
                const int h = max(__hip_atomic_load(&A.helpers[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), 0);
                ok = rem > 0 && (h == 0 || rem >= (long long)(h + 1) * A.share);
            }
            const unsigned long long m = __ballot(ok);
            if (m) return A.order[b + __ffsll((unsigned long long)m) - 1];
        }
    } else {
        for (int b = 0; b < A.n_order; b += 64) {
            const int i = b + lane;
            bool fresh = false;
            if (i < A.n_order) {
                const int r = A.order[i];
                fresh = !A.reqs[r].retired &&
                        __hip_atomic_load(&A.next[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0ull;
            }
            const unsigned long long m = __ballot(fresh);
            if (m) return A.order[b + __ffsll((unsigned long long)m) - 1];
        }
    }
    // every request is open: help the one with the most unclaimed trajectories
    long long best = 0;
    int bi = -1;
    for (int b = 0; b < A.n_order; b += 64) {
        const int i = b + lane;
        const long long rem = i < A.n_order ? remaining_of(A, A.order[i]) : 0;
        if (rem > best) {
            best = rem;
            bi = i;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const long long ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi >= 0 && (bi < 0 || oi < bi))) {
            best = ob;
            bi = oi;
        }
    }
    return best > 0 ? A.order[bi] : -1;
}

// Called by a whole wavefront (all 64 lanes converged) when the lanes in
// `mask` need work.  On return a lane in `mask` either has a trajectory
// (req >= 0, queue position pos, table slot slot) or req = -1.
// load(slot, r) copies request r's table into a slot with the wave's lanes.
template <int SLOTS, class Load>
__device__ __forceinline__ void wave_acquire(WgSched &S, const SliceArgs &A, unsigned long long mask,
                                             int &req, long long &pos, int &slot, Load &&load)
{
    const int lane = __lane_id();
    req = -1;
    int got = 0;
    if (lane == 0) {
        int expected = 0;
        got = __hip_atomic_compare_exchange_strong(&S.lock, &expected, 1, __ATOMIC_ACQUIRE,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    got = __shfl(got, 0);
    if (!got) return;   // another wave is scheduling; try again next iteration

    int cur = __shfl(S.cur, 0);
    int r = __shfl(S.slot_req[cur], 0);
    const int dry = __shfl(S.dry, 0);
    const int done = __shfl(S.done, 0);
    if ((r < 0 || dry) && !done) {
        const int other = SLOTS == 2 ? cur ^ 1 : cur;
        const int busy = __hip_atomic_load(&S.active[other], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int leaving = r;   // the request this workgroup has drawn from (or -1)
        r = -1;
        if (__shfl(busy, 0) == 0) {
            const int nr = pick_request(A);
            if (nr < 0) {
                if (lane == 0) S.done = 1;
            } else {
                if (__shfl(S.slot_req[other], 0) != nr) load(other, nr);
                if (lane == 0 && A.helpers) {
                    // this workgroup now draws from nr instead of the request it leaves
                    if (leaving >= 0)
                        __hip_atomic_fetch_add(&A.helpers[leaving], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_add(&A.helpers[nr], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (lane == 0) {
                    S.slot_req[other] = nr;
                    S.cur = other;
                    S.dry = 0;
                }
                cur = other;
                r = nr;
            }
        }
    } else if (dry) {
        r = -1;
    }
    if (r >= 0) {
        const long long nt = A.reqs[r].P.n_traj;
        const int n = __popcll(mask);
        unsigned long long p0 = 0;
        if (lane == 0) p0 = atomicAdd(&A.next[r], (unsigned long long)n);
        p0 = __shfl(p0, 0);
        long long k = nt - (long long)p0;
        k = k < 0 ? 0 : (k > n ? n : k);
        if (lane == 0) {
            if ((long long)p0 + n >= nt) S.dry = 1;
            if (k > 0)
                __hip_atomic_fetch_add(&S.active[cur], (int)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (((mask >> lane) & 1ull) && rank < k) {
            req = r;
            pos = (long long)p0 + rank;
            slot = cur;
        }
    }
    if (lane == 0) __hip_atomic_store(&S.lock, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A lane finished (or dropped) a trajectory drawn from `slot`.
__device__ __forceinline__ void slot_release(WgSched &S, int slot)
{
    __hip_atomic_fetch_add(&S.active[slot], -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Thread 0: scheduling state at the start of a launch.
__device__ __forceinline__ void sched_init(WgSched &S, const SliceArgs &A)
{
    S.slot_req[0] = S.slot_req[1] = -1;
    S.active[0] = S.active[1] = 0;
    S.cur = 0;
    S.dry = 1;
    S.lock = 0;
    S.done = 0;
    if (A.resume && A.wg_save) {
        const WgSave w = A.wg_save[blockIdx.x];
        for (int s = 0; s < 2; ++s) {
            const int r = w.slot_req[s];
            S.slot_req[s] = (r >= 0 && !A.reqs[r].retired) ? r : -1;
        }
        S.cur = w.cur & 1;
        if (S.slot_req[S.cur] < 0 && S.slot_req[S.cur ^ 1] < 0) S.cur = 0;
        S.dry = S.slot_req[S.cur] < 0;
    }
}

}  // namespace nh
