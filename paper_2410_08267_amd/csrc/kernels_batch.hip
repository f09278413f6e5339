// Slice kernels of the batched and serving forms (FP64 and FP32-compensated)
// and the reductions over many requests.
//
// Every lane runs the same per-trajectory code as the plain kernels (start,
// Dormand-Prince attempt, outputs); only the source of its request parameters
// differs: a descriptor in HBM and one of the workgroup's two LDS table slots
// (see nh_batch.h for the scheduling).
#include <hip/hip_runtime.h>

#include "nh_batch.h"
#include "nh_dp5_f32.h"
#include "nh_launch.h"
#include "nh_reduce.h"

namespace nh {

// FP64 coefficients from rows of STRIDE doubles of which the first NC columns
// are interpolated; R comes from its column for requests with a moving
// compensation radius (nc == NCOL, possible only when NC == NCOL), else it is
// the request's constant.  HIST: launches holding requests with non-smooth
// histories keep each request's stencils inside its spline pieces (Knots) and
// apply its power-law factor of K and Kc (PowFactor); for smooth requests both
// leave the values unchanged bit for bit (one piece, factor exactly 1).
template <int NC, int STRIDE = NC, bool HIST = false, bool PAIRED = false>
struct TabCoefB {
    const double *tab;
    int nc, n_tab;
    double u0, inv_du, R_const;
    PowFactor pw;
    Knots kn;
    __device__ __forceinline__ void at(double u, double c[NCOL], double &R) const
    {
        coef_interp<NC, STRIDE, HIST>(tab, n_tab, u0, inv_du, kn, u, c);
        R = (NC == NCOL && nc == NCOL) ? c[COL_R] : R_const;
        if constexpr (HIST) {
            const double f = pow_factor(pw, u);
            c[COL_K] *= f;
            c[COL_KC] *= f;
        }
    }
    // PAIRED: stages 2 and 3 share one five-row window, as in the plain
    // kernel (same values bit for bit); otherwise four rows per stage, where
    // the window's registers are not available
    static constexpr bool paired = PAIRED;
    __device__ __forceinline__ void at2(double uP, double uQ, double cP[NCOL], double &RP, double cQ[NCOL],
                                        double &RQ) const
    {
        static_assert(!HIST, "paired window only for smooth histories");
        coef_interp2<NC, STRIDE, HIST>(tab, n_tab, u0, inv_du, kn, uP, uQ, cP, cQ);
        RP = (NC == NCOL && nc == NCOL) ? cP[COL_R] : R_const;
        RQ = (NC == NCOL && nc == NCOL) ? cQ[COL_R] : R_const;
    }
};

// Copy request q's table into a slot: FP64 rows of NC doubles (NC of the
// staged NCOL columns), or the FP32C layout (stage_f32c_table), by the threads
// first, first + step, ...
template <int NC>
__device__ __forceinline__ void copy_table(double *dst, const BatchReq &q, int first, int step)
{
    const int n = q.P.n_tab * NC;
    const double *src = q.g.tab;
    for (int i = first; i < n; i += step) {
        const int node = i / NC, col = i - node * NC;
        dst[i] = src[node * NCOL + col];
    }
}

// The plain kernel's split layout in a slot of n_tab rows of SPLIT_ROW
// doubles: K, Kc, 1/s and c (the drift column A is read from the request's
// staged copy in device memory).
__device__ __forceinline__ void copy_table_split(double *dst, const BatchReq &q, int first, int step)
{
    const int n = q.P.n_tab * 4;
    const double *src = q.g.tab;
    for (int i = first; i < n; i += step) {
        const int node = i >> 2, col = i & 3;
        dst[node * SPLIT_ROW + col] = src[node * NCOL + COL_K + col];
    }
}

// Bytes of one FP32C table slot (kept a multiple of 16 so the next slot's
// FP64 rows stay aligned).
template <int NC>
__host__ __device__ constexpr size_t f32c_slot_bytes(int n_tab)
{
    return (f32c_table_bytes<NC>(n_tab) + 15) & ~(size_t)15;
}

// Initial position and velocity of trajectory t = (k n_y + j) n_mu + l.
__device__ __forceinline__ void initial_state(const BatchReq &q, long long t, double &x0, double &vx0,
                                              double &vy0)
{
    const TrajParams &P = q.P;
    const TrajIdx ix = traj_idx(t, P);
    const int l = ix.l, j = ix.j, k = ix.k;
    const double V = q.g.y[j] * P.vfac;
    vx0 = V * q.g.mu[l];
    vy0 = V * q.g.smu[l];
    x0 = q.g.r[k];
}

__device__ __forceinline__ void finish_free(const BatchReq &q, long long t)
{
    q.o.ratio[t] = 1.0;
    q.o.stat[t] = TrajStat{0, 0, ST_OK | ST_FREE_EXIT, 0};
}

__device__ __forceinline__ unsigned long long pack2f(float a, float b)
{
    return ((unsigned long long)__float_as_uint(a) << 32) | __float_as_uint(b);
}
__device__ __forceinline__ unsigned long long pack2i(int a, int b)
{
    return ((unsigned long long)(unsigned)a << 32) | (unsigned)b;
}
__device__ __forceinline__ float hi_f(unsigned long long w) { return __uint_as_float((unsigned)(w >> 32)); }
__device__ __forceinline__ float lo_f(unsigned long long w) { return __uint_as_float((unsigned)w); }
__device__ __forceinline__ int hi_i(unsigned long long w) { return (int)(unsigned)(w >> 32); }
__device__ __forceinline__ int lo_i(unsigned long long w) { return (int)(unsigned)w; }
__device__ __forceinline__ unsigned long long bits(double d) { return (unsigned long long)__double_as_longlong(d); }
__device__ __forceinline__ double dbl(unsigned long long w) { return __longlong_as_double((long long)w); }

__device__ __forceinline__ void pack64(const Lane64 &L, double v0n, LaneSave &s)
{
    s.w[0] = bits(L.x);
    s.w[1] = bits(L.y);
    s.w[2] = bits(L.vx);
    s.w[3] = bits(L.vy);
    s.w[4] = bits(L.u);
    s.w[5] = bits(L.h);
    s.w[6] = bits(L.k1x);
    s.w[7] = bits(L.k1y);
    s.w[8] = bits(L.k1u);
    s.w[9] = bits(L.k1v);
    s.w[10] = bits(v0n);
    s.w[11] = pack2i(L.nacc, L.nrej);
    s.w[12] = pack2i(L.natt, L.rej_prev ? 1 : 0);
}
__device__ __forceinline__ void unpack64(const LaneSave &s, Lane64 &L, double &v0n)
{
    L.x = dbl(s.w[0]);
    L.y = dbl(s.w[1]);
    L.vx = dbl(s.w[2]);
    L.vy = dbl(s.w[3]);
    L.u = dbl(s.w[4]);
    L.h = dbl(s.w[5]);
    L.k1x = dbl(s.w[6]);
    L.k1y = dbl(s.w[7]);
    L.k1u = dbl(s.w[8]);
    L.k1v = dbl(s.w[9]);
    v0n = dbl(s.w[10]);
    L.nacc = hi_i(s.w[11]);
    L.nrej = lo_i(s.w[11]);
    L.natt = hi_i(s.w[12]);
    L.rej_prev = lo_i(s.w[12]) != 0;
}

__device__ __forceinline__ void pack32(const Lane32 &L, double v0n, LaneSave &s)
{
    s.w[0] = pack2f(L.x, L.y);
    s.w[1] = pack2f(L.xc, L.yc);
    s.w[2] = pack2f(L.vx, L.vy);
    s.w[3] = bits(L.u);
    s.w[4] = bits(L.h);
    s.w[5] = pack2f(L.k1x, L.k1y);
    s.w[6] = pack2f(L.k1u, L.k1v);
    s.w[7] = bits(v0n);
    s.w[8] = pack2i(L.nacc, L.nrej);
    s.w[9] = pack2i(L.natt, L.n64);
    s.w[10] = L.rej_prev ? 1ull : 0ull;
}
__device__ __forceinline__ void unpack32(const LaneSave &s, Lane32 &L, double &v0n)
{
    L.x = hi_f(s.w[0]);
    L.y = lo_f(s.w[0]);
    L.xc = hi_f(s.w[1]);
    L.yc = lo_f(s.w[1]);
    L.vx = hi_f(s.w[2]);
    L.vy = lo_f(s.w[2]);
    L.u = dbl(s.w[3]);
    L.h = dbl(s.w[4]);
    L.k1x = hi_f(s.w[5]);
    L.k1y = lo_f(s.w[5]);
    L.k1u = hi_f(s.w[6]);
    L.k1v = lo_f(s.w[6]);
    v0n = dbl(s.w[7]);
    L.nacc = hi_i(s.w[8]);
    L.nrej = lo_i(s.w[8]);
    L.natt = hi_i(s.w[9]);
    L.n64 = lo_i(s.w[9]);
    L.rej_prev = s.w[10] != 0ull;
}

// Per-lane parameters of a trajectory of request q whose table sits in `slot`.
template <int NC, bool HIST, bool PAIRED = false>
struct Lane64Params {
    TabCoefB<NC, NC, HIST, PAIRED> cf;
    DpCtl ctl;
};
template <int NC, bool HIST, bool PAIRED>
__device__ __forceinline__ void setup64(const BatchReq &q, const double *slot, Lane64Params<NC, HIST, PAIRED> &p)
{
    const TrajParams &P = q.P;
    p.cf = TabCoefB<NC, NC, HIST, PAIRED>{slot, q.nc, P.n_tab, P.tab_u0, P.tab_inv_du, P.R_const, P.pw, P.kn};
    p.ctl.u_end = P.u_end;
    p.ctl.rtol = P.rtol;
    p.ctl.atol_x = P.atol_x;
    p.ctl.atol_v = P.atol_v;
    p.ctl.r_exit2 = P.r_exit2;
    p.ctl.max_steps = (int)P.max_steps;
}

// The same from a wave-uniform request index, through the constant address
// space: descriptors do not change while a kernel runs, so these are scalar
// loads into scalar registers (through a generic pointer the compiler cannot
// rule out the kernel's own stores and loads them per lane).  Smooth
// histories only: the spline pieces and factors are not read.
using ConstReq = const __attribute__((address_space(4))) BatchReq;
template <int NC, bool PAIRED>
__device__ __forceinline__ void setup64_uniform(const BatchReq *reqs, int ru, const double *slot,
                                                Lane64Params<NC, false, PAIRED> &p)
{
    ConstReq *q = (ConstReq *)(reqs + ru);
    p.cf.tab = slot;
    p.cf.nc = q->nc;
    p.cf.n_tab = q->P.n_tab;
    p.cf.u0 = q->P.tab_u0;
    p.cf.inv_du = q->P.tab_inv_du;
    p.cf.R_const = q->P.R_const;
    p.ctl.u_end = q->P.u_end;
    p.ctl.rtol = q->P.rtol;
    p.ctl.atol_x = q->P.atol_x;
    p.ctl.atol_v = q->P.atol_v;
    p.ctl.r_exit2 = q->P.r_exit2;
    p.ctl.max_steps = (int)q->P.max_steps;
}

// Five-column launches with one slot and smooth histories: the split table
// (as the plain kernel: a fifth of the table reads off the LDS) with the
// parameters as scalars, same values bit for bit.
template <int NC, int SLOTS, bool HIST>
constexpr bool slice_split = NC == SPLIT_ROW && SLOTS == 1 && !HIST;
struct SplitParams {
    TabCoefSplit<false> cf;
    DpCtl ctl;
};
__device__ __forceinline__ void setup_split_uniform(const BatchReq *reqs, int ru, const double *slot, SplitParams &p)
{
    ConstReq *q = (ConstReq *)(reqs + ru);
    p.cf.lds = slot;
    p.cf.a = q->g.tabA;
    p.cf.n_tab = q->P.n_tab;
    p.cf.u0 = q->P.tab_u0;
    p.cf.inv_du = q->P.tab_inv_du;
    p.cf.R_const = q->P.R_const;
    p.ctl.u_end = q->P.u_end;
    p.ctl.rtol = q->P.rtol;
    p.ctl.atol_x = q->P.atol_x;
    p.ctl.atol_v = q->P.atol_v;
    p.ctl.r_exit2 = q->P.r_exit2;
    p.ctl.max_steps = (int)q->P.max_steps;
}

// A request descriptor read with a wave-uniform index through the constant
// address space, word by word into a local copy (only the words used are
// loaded): scalar loads into scalar registers.  Descriptors do not change
// while a kernel runs; through a generic pointer the compiler cannot rule out
// the kernel's own stores and loads them per lane.
__device__ __forceinline__ BatchReq load_uniform(const BatchReq *p)
{
    static_assert(sizeof(BatchReq) % 4 == 0, "descriptor words");
    constexpr int N = (int)(sizeof(BatchReq) / 4);
    using W = const __attribute__((address_space(4))) unsigned;
    W *w = (W *)p;
    unsigned buf[N];
#pragma unroll
    for (int i = 0; i < N; ++i) buf[i] = w[i];
    BatchReq q;
    __builtin_memcpy(&q, buf, sizeof(BatchReq));
    return q;
}

// SPLIT: the table slot holds the split FP32C layout (K, Kc in FP64; A from
// the request's staged copy in device memory), with the shared window of
// stages 2 and 3.
template <int NC, bool HIST, bool SPLIT = false>
struct Lane32Params {
    TabCoef32<NC, HIST, SPLIT> cf;
    TabCoefB<NC, NCOL, HIST> cf64;    // the promoted FP64 attempts read the FP64 table from HBM
    DpCtl32 ctl;
    DpCtl ctl64;
    double h_fp64;
};
template <int NC, bool HIST, bool SPLIT>
__device__ __forceinline__ void setup32(const BatchReq &q, const char *slot, Lane32Params<NC, HIST, SPLIT> &p)
{
    const TrajParams &P = q.P;
    const double *t64 = (const double *)slot;
    p.cf = TabCoef32<NC, HIST, SPLIT>{t64, (const float *)(t64 + (size_t)P.n_tab * f32c_t64<SPLIT>), q.nc,
                                     P.n_tab, P.tab_u0, P.tab_inv_du, (float)fmin(P.R_const, 1.0e30), P.pw,
                                     P.kn, q.g.tabA};
    p.cf64 = TabCoefB<NC, NCOL, HIST>{q.g.tab, q.nc, P.n_tab, P.tab_u0, P.tab_inv_du, P.R_const, P.pw, P.kn};
    f32c_controls(P, p.ctl, p.ctl64);
    p.h_fp64 = P.h_fp64;
}

// ---------------------------------------------------------------------------
// FP64 slice kernel
// ---------------------------------------------------------------------------

// FP64 slices run up to 1024 threads per workgroup (four waves per SIMD); the
// FP32-compensated lane state needs more than the 128 VGPRs that allows.
template <int NC, int SLOTS, bool HIST>
__global__ __launch_bounds__(1024) void k_slice_f64(SliceArgs A)
{
    extern __shared__ double lds64[];
    __shared__ WgSched S;
    const int slot_n = A.n_tab * NC;
    if (threadIdx.x == 0) sched_init(S, A);
    __syncthreads();
    constexpr bool SPLIT = slice_split<NC, SLOTS, HIST>;
    for (int s = 0; s < SLOTS; ++s)
        if (S.slot_req[s] >= 0) {
            if constexpr (SPLIT) copy_table_split(lds64 + s * slot_n, A.reqs[S.slot_req[s]], threadIdx.x, blockDim.x);
            else copy_table<NC>(lds64 + s * slot_n, A.reqs[S.slot_req[s]], threadIdx.x, blockDim.x);
        }

    long long t = -1;
    int rq = 0, sl = 0;
    double v0n = 1.0;
    Lane64 L{};
    Lane64Params<NC, HIST> lp{};
    // this lane's save record (recomputed where used rather than held in
    // registers through the loop)
    const auto my_save = [&]() { return A.lane_save + ((size_t)blockIdx.x * blockDim.x + threadIdx.x); };
    if (A.resume && A.lane_save) {
        const LaneSave sv = *my_save();
        if (sv.t >= 0 && !A.reqs[sv.req].retired) {
            t = sv.t;
            rq = sv.req;
            sl = SLOTS == 1 ? 0 : sv.slot;
            unpack64(sv, L, v0n);
            setup64(A.reqs[rq], lds64 + sl * slot_n, lp);
            __hip_atomic_fetch_add(&S.active[sl], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();

    const unsigned long long t0 = wall_clock64();
    bool expired = false;
    for (;;) {
        if (A.budget_ticks >= 0 && !expired) expired = (long long)(wall_clock64() - t0) > A.budget_ticks;
        const unsigned long long mask = __ballot(t < 0 && !expired);
        if (mask != 0ull && !__hip_atomic_load(&S.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            int r, s;
            long long p;
            wave_acquire<SLOTS>(S, A, mask, r, p, s, [&](int slot, int req) {
                if constexpr (SPLIT) copy_table_split(lds64 + slot * slot_n, A.reqs[req], (int)__lane_id(), 64);
                else copy_table<NC>(lds64 + slot * slot_n, A.reqs[req], (int)__lane_id(), 64);
            });
            if (r >= 0) {
                // the lanes that got a trajectory share one request and slot
                const int ru = __builtin_amdgcn_readfirstlane(r);
                const BatchReq &q = A.reqs[ru];
                rq = ru;
                sl = SLOTS == 1 ? 0 : s;
                t = traj_of(p, q.P);
                if (q.free_all) {
                    finish_free(q, t);
                    slot_release(S, sl);
                    t = -1;
                } else {
                    double x0, vx0, vy0;
                    initial_state(q, t, x0, vx0, vy0);
                    v0n = sqrt(norm2(vx0, vy0));
                    if (q.P.cull_D > 0.0 && never_enters(x0, vx0, vy0, q.P.cull_D, cull_radius2(q.P.r_exit))) {
                        finish_free(q, t);
                        slot_release(S, sl);
                        t = -1;
                    } else if constexpr (SPLIT) {
                        SplitParams up;
                        setup_split_uniform(A.reqs, ru, lds64, up);
                        dp5_start(L, up.cf, x0, vx0, vy0, q.P.h0, q.P.u_start, q.P.u_end);
                    } else if constexpr (SLOTS == 1 && !HIST) {
                        Lane64Params<NC, HIST, true> up;
                        setup64_uniform(A.reqs, ru, lds64, up);
                        dp5_start(L, up.cf, x0, vx0, vy0, q.P.h0, q.P.u_start, q.P.u_end);
                    } else {
                        setup64(q, lds64 + sl * slot_n, lp);
                        dp5_start(L, lp.cf, x0, vx0, vy0, q.P.h0, q.P.u_start, q.P.u_end);
                    }
                }
            }
        }
        if (__ballot(t >= 0) == 0ull) {
            if (expired || __hip_atomic_load(&S.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        if (expired) break;
        if (t >= 0) {
            int st;
            if constexpr (SPLIT) {
                SplitParams up;
                setup_split_uniform(A.reqs, __builtin_amdgcn_readfirstlane(rq), lds64, up);
                st = dp5_attempt(L, up.cf, up.ctl);
            } else if constexpr (SLOTS == 1 && !HIST) {
                // With one slot a workgroup loads a new request only once no
                // lane runs a trajectory of the old one, so every lane here
                // serves the same request: its parameters are wave-uniform and
                // come through scalar loads instead of lane registers, which
                // leaves room for the shared window of stages 2 and 3.  (The
                // spline pieces and factors of sampled histories would not fit
                // the scalar registers.)
                Lane64Params<NC, HIST, true> up;
                setup64_uniform(A.reqs, __builtin_amdgcn_readfirstlane(rq), lds64, up);
                st = dp5_attempt(L, up.cf, up.ctl);
            } else {
                st = dp5_attempt(L, lp.cf, lp.ctl);
            }
            if (st >= 0) {
                const TrajOut o = A.reqs[rq].o;
                o.ratio[t] = sqrt(norm2(L.vx, L.vy)) / v0n;
                o.stat[t] = TrajStat{L.nacc, L.nrej, st, 0};
                slot_release(S, sl);
                t = -1;
            }
        }
    }
    if (A.lane_save) {
        LaneSave sv;
        sv.t = t;
        sv.req = rq;
        sv.slot = sl;
        if (t >= 0) {
            pack64(L, v0n, sv);
            atomicAdd(&A.inflight[rq], 1u);
        }
        *my_save() = sv;
    }
    __syncthreads();
    if (threadIdx.x == 0 && A.wg_save) A.wg_save[blockIdx.x] = WgSave{{S.slot_req[0], S.slot_req[1]}, S.cur, 0};
}

// ---------------------------------------------------------------------------
// FP32-compensated slice kernel
// ---------------------------------------------------------------------------

// Two slots: at most 768 threads (three waves per SIMD: the lane state with
// per-lane request parameters needs ~160 VGPRs).  One slot: 1024 (four waves;
// with smooth histories the request parameters sit in scalar registers, and
// the sampled-history variant spills a few values).
template <int NC, int SLOTS, bool HIST>
constexpr int f32c_slice_max_block = SLOTS == 1 ? 1024 : 768;
template <int NC, int SLOTS, bool HIST>
__global__ __launch_bounds__((f32c_slice_max_block<NC, SLOTS, HIST>)) void k_slice_f32c(SliceArgs A)
{
    extern __shared__ double lds32b[];
    __shared__ WgSched S;
    char *const slots = (char *)lds32b;
    const size_t slot_n = f32c_slot_bytes<NC>(A.n_tab);
    // one slot, smooth histories: every lane running a trajectory serves the
    // slot's one request (a new one is loaded only once none runs), so its
    // parameters are wave-uniform scalars, which leaves registers for the
    // split table and the shared window of stages 2 and 3
    constexpr bool UNI = SLOTS == 1 && !HIST;
    if (threadIdx.x == 0) sched_init(S, A);
    __syncthreads();
    for (int s = 0; s < SLOTS; ++s)
        if (S.slot_req[s] >= 0)
            stage_f32c_table<NC, UNI>(slots + s * slot_n, A.reqs[S.slot_req[s]].g.tab,
                                      A.reqs[S.slot_req[s]].P.n_tab, threadIdx.x, blockDim.x);

    long long t = -1;
    int rq = 0, sl = 0;
    double v0n = 1.0;
    Lane32 L{};
    Lane32Params<NC, HIST> lp{};
    const auto my_save = [&]() { return A.lane_save + ((size_t)blockIdx.x * blockDim.x + threadIdx.x); };
    if (A.resume && A.lane_save) {
        const LaneSave sv = *my_save();
        if (sv.t >= 0 && !A.reqs[sv.req].retired) {
            t = sv.t;
            rq = sv.req;
            sl = SLOTS == 1 ? 0 : sv.slot;
            unpack32(sv, L, v0n);
            setup32(A.reqs[rq], slots + sl * slot_n, lp);
            __hip_atomic_fetch_add(&S.active[sl], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();

    const unsigned long long t0 = wall_clock64();
    bool expired = false;
    for (;;) {
        if (A.budget_ticks >= 0 && !expired) expired = (long long)(wall_clock64() - t0) > A.budget_ticks;
        const unsigned long long mask = __ballot(t < 0 && !expired);
        if (mask != 0ull && !__hip_atomic_load(&S.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            int r, s;
            long long p;
            wave_acquire<SLOTS>(S, A, mask, r, p, s, [&](int slot, int req) {
                stage_f32c_table<NC, UNI>(slots + slot * slot_n, A.reqs[req].g.tab, A.reqs[req].P.n_tab,
                                          (int)__lane_id(), 64);
            });
            if (r >= 0) {
                // the lanes that got a trajectory share one request and slot
                const int ru = __builtin_amdgcn_readfirstlane(r);
                const BatchReq &q = A.reqs[ru];
                rq = ru;
                sl = SLOTS == 1 ? 0 : s;
                t = traj_of(p, q.P);
                if (q.free_all) {
                    finish_free(q, t);
                    slot_release(S, sl);
                    t = -1;
                } else {
                    double x0, vx0, vy0;
                    initial_state(q, t, x0, vx0, vy0);
                    v0n = sqrt(norm2(vx0, vy0));
                    if (q.P.cull_D > 0.0 && never_enters(x0, vx0, vy0, q.P.cull_D, cull_radius2(q.P.r_exit))) {
                        finish_free(q, t);
                        slot_release(S, sl);
                        t = -1;
                    } else if constexpr (UNI) {
                        Lane32Params<NC, false, true> up;
                        setup32(load_uniform(A.reqs + ru), slots, up);
                        f32c_start(L, up.cf, x0, vx0, vy0, q.P.h0, q.P.u_start, q.P.u_end);
                    } else {
                        setup32(q, slots + sl * slot_n, lp);
                        f32c_start(L, lp.cf, x0, vx0, vy0, q.P.h0, q.P.u_start, q.P.u_end);
                    }
                }
            }
        }
        if (__ballot(t >= 0) == 0ull) {
            if (expired || __hip_atomic_load(&S.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        if (expired) break;
        if (t >= 0) {
            int st;
            if constexpr (UNI) {
                Lane32Params<NC, false, true> up;
                setup32(load_uniform(A.reqs + __builtin_amdgcn_readfirstlane(rq)), slots, up);
                st = f32c_attempt(L, up.cf, up.cf64, up.ctl, up.ctl64, up.h_fp64);
            } else {
                st = f32c_attempt(L, lp.cf, lp.cf64, lp.ctl, lp.ctl64, lp.h_fp64);
            }
            if (st >= 0) {
                const TrajOut o = A.reqs[rq].o;
                const double fx = L.vx, fy = L.vy;
                o.ratio[t] = sqrt(norm2(fx, fy)) / v0n;
                o.stat[t] = TrajStat{L.nacc, L.nrej, st, L.n64};
                slot_release(S, sl);
                t = -1;
            }
        }
    }
    if (A.lane_save) {
        LaneSave sv;
        sv.t = t;
        sv.req = rq;
        sv.slot = sl;
        if (t >= 0) {
            pack32(L, v0n, sv);
            atomicAdd(&A.inflight[rq], 1u);
        }
        *my_save() = sv;
    }
    __syncthreads();
    if (threadIdx.x == 0 && A.wg_save) A.wg_save[blockIdx.x] = WgSave{{S.slot_req[0], S.slot_req[1]}, S.cur, 0};
}

// ---------------------------------------------------------------------------
// reductions over listed requests
// ---------------------------------------------------------------------------

// One block per radius of the listed requests; rstart[i] = first block of list[i].
__global__ __launch_bounds__(256) void k_reduce_profile_batch(const BatchReq *__restrict__ reqs,
                                                              const int *__restrict__ list,
                                                              const int *__restrict__ rstart, int n_list)
{
    const int b = blockIdx.x;
    int lo = 0, hi = n_list - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rstart[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const BatchReq &q = reqs[list[lo]];
    reduce_radius(q.P, q.g, q.o.ratio, b - rstart[lo], q.out);
}

// blockIdx.y: listed request; its statistics go to stats[8 * blockIdx.y ...].
__global__ __launch_bounds__(256) void k_reduce_stats_batch(const BatchReq *__restrict__ reqs,
                                                            const int *__restrict__ list,
                                                            unsigned long long *stats)
{
    const BatchReq &q = reqs[list[blockIdx.y]];
    reduce_stats_range(q.o.stat, (long long)blockIdx.x * blockDim.x + threadIdx.x, q.P.n_traj,
                       (long long)gridDim.x * blockDim.x, stats + 8 * (size_t)blockIdx.y);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

size_t slice_lds_bytes(bool f32c, int nc, int slots, int n_tab)
{
    if (f32c)
        return (size_t)slots * (nc == NCOL ? f32c_slot_bytes<NCOL>(n_tab) : f32c_slot_bytes<NCOL - 1>(n_tab));
    return (size_t)slots * n_tab * nc * sizeof(double);
}

int slice_max_table_nodes(bool f32c, int nc, int slots)
{
    const size_t avail = 160 * 1024 - sizeof(WgSched) - 256;
    const size_t per_node = f32c ? F32C_T64 * sizeof(double) + (nc - F32C_T64) * sizeof(float) : nc * sizeof(double);
    // one node of slack per slot for the alignment of the next slot
    return (int)(avail / ((size_t)slots * per_node)) - 1;
}

template <int NC, int SLOTS, bool HIST>
static const void *slice_fn(bool f32c)
{
    return f32c ? (const void *)k_slice_f32c<NC, SLOTS, HIST> : (const void *)k_slice_f64<NC, SLOTS, HIST>;
}

template <bool HIST>
static const void *slice_fn_hist(bool f32c, int nc, int slots)
{
    if (nc == NCOL) return slots == 2 ? slice_fn<NCOL, 2, HIST>(f32c) : slice_fn<NCOL, 1, HIST>(f32c);
    return slots == 2 ? slice_fn<NCOL - 1, 2, HIST>(f32c) : slice_fn<NCOL - 1, 1, HIST>(f32c);
}

static const void *slice_fn(bool f32c, int nc, int slots, bool pow)
{
    return pow ? slice_fn_hist<true>(f32c, nc, slots) : slice_fn_hist<false>(f32c, nc, slots);
}

// Workgroups that fit the device at once for this slice configuration.
hipError_t slice_capacity(bool f32c, int nc, int slots, bool pow, int n_tab, int block, int n_cu, int *grid)
{
    const void *fn = slice_fn(f32c, nc, slots, pow);
    const size_t lds = slice_lds_bytes(f32c, nc, slots, n_tab);
    int per_cu = 0;
    const hipError_t e = occupancy_cached(fn, block, lds, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    *grid = n_cu * per_cu;
    return hipSuccess;
}

hipError_t launch_slice(const SliceArgs &A, bool f32c, int nc, int slots, bool pow, int grid, int block,
                        hipStream_t s)
{
    const size_t lds = slice_lds_bytes(f32c, nc, slots, A.n_tab);
    void *args[] = {(void *)&A};
    return hipLaunchKernel(slice_fn(f32c, nc, slots, pow), dim3(grid), dim3(block), args, lds, s);
}

// One serving slice as a graph: upload the descriptors and the run order,
// clear the in-flight counts (a kernel, not a memset node), run the slice
// kernel, bring back the queue positions and in-flight counts.  The slice
// kernel's arguments change every slice and are set on the instantiated graph
// before each launch (slice_graph_launch).
hipError_t slice_graph_build(SliceGraph &G, const SliceGraphBufs &b, const SliceArgs &A, bool f32c, int nc,
                             int slots, bool pow, int grid, int block)
{
    slice_graph_destroy(G);
    hipError_t e = hipGraphCreate(&G.graph, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t up_desc, up_order, clear, back_next, back_inflight;
    if ((e = hipGraphAddMemcpyNode1D(&up_desc, G.graph, nullptr, 0, b.d_desc, b.h_desc, b.desc_bytes,
                                     hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if ((e = hipGraphAddMemcpyNode1D(&up_order, G.graph, nullptr, 0, b.d_order, b.h_order, b.order_bytes,
                                     hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    unsigned long long *p = (unsigned long long *)b.d_inflight;
    int n = (int)(b.inflight_bytes / sizeof(unsigned long long));
    unsigned long long zero = 0ull;
    void *fill_args[] = {(void *)&p, (void *)&n, (void *)&zero};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(fill_u64_kernel());
    kp.gridDim = dim3((unsigned)((n + 255) / 256));
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = fill_args;
    if ((e = hipGraphAddKernelNode(&clear, G.graph, nullptr, 0, &kp)) != hipSuccess) return e;
    G.args = A;
    G.params = hipKernelNodeParams{};
    G.params.func = const_cast<void *>(slice_fn(f32c, nc, slots, pow));
    G.params.gridDim = dim3(grid);
    G.params.blockDim = dim3(block);
    G.params.sharedMemBytes = (unsigned)slice_lds_bytes(f32c, nc, slots, A.n_tab);
    G.arg_ptr[0] = (void *)&G.args;
    G.params.kernelParams = G.arg_ptr;
    hipGraphNode_t deps[3] = {up_desc, up_order, clear};
    if ((e = hipGraphAddKernelNode(&G.slice, G.graph, deps, 3, &G.params)) != hipSuccess) return e;
    if ((e = hipGraphAddMemcpyNode1D(&back_next, G.graph, &G.slice, 1, b.h_next, b.d_next, b.next_bytes,
                                     hipMemcpyDeviceToHost)) != hipSuccess)
        return e;
    if ((e = hipGraphAddMemcpyNode1D(&back_inflight, G.graph, &G.slice, 1, b.h_inflight, b.d_inflight,
                                     b.inflight_bytes, hipMemcpyDeviceToHost)) != hipSuccess)
        return e;
    if ((e = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0)) != hipSuccess) return e;
    G.f32c = f32c;
    G.nc = nc;
    G.slots = slots;
    G.pow = pow;
    G.grid = grid;
    G.block = block;
    return hipSuccess;
}

hipError_t slice_graph_launch(SliceGraph &G, const SliceArgs &A, hipStream_t s)
{
    G.args = A;
    G.params.kernelParams = G.arg_ptr;
    hipError_t e = hipGraphExecKernelNodeSetParams(G.exec, G.slice, &G.params);
    if (e != hipSuccess) return e;
    return hipGraphLaunch(G.exec, s);
}

void slice_graph_destroy(SliceGraph &G)
{
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    G.exec = nullptr;
    G.graph = nullptr;
    G.slice = nullptr;
    G.nc = 0;
}

hipError_t launch_reduce_batch(const BatchReq *reqs, const int *list, const int *rstart, int n_list,
                               int n_blocks, unsigned long long *stats, int stat_chunks, hipStream_t s)
{
    if (n_list <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_profile_batch, dim3(n_blocks), dim3(256), 0, s, reqs, list, rstart, n_list);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_stats_batch, dim3(stat_chunks, n_list), dim3(256), 0, s, reqs, list, stats);
    return hipGetLastError();
}

}  // namespace nh
