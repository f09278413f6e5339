#!/usr/bin/env python3
"""Benchmark: n(r)/nbar profiles of relics around a time-evolving NFW halo.

One step = one full profile of the plain-at-scale workload (100 radii x 200 |p|
x 64 cos(psi) = 1.28 M trajectories, Dormand-Prince 5(4) at rtol 1e-8, FP64,
z 0 -> 4), a different seeded halo per step (seeds 0..K-1; warm-up uses
seeds 1000+).  Inputs are the request descriptors; every step stages its FP64
tables and grids (~150 kB) to HBM, integrates every trajectory and adds each
one's quadrature term to the profile on the GPU.

Prints one JSON line.  value = accepted trajectory steps per second over the
timed steps.  roofline: the trajectory kernel's algorithmic FP64 FLOP rate
against the MI355X FP64 vector peak.  cpu_baseline: the CPU oracle on the
seed-0 profile, on this host's cores; the same leg compares the GPU's profiles
with the oracle's (max_rel_err_vs_oracle).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 FLOP of one attempted Dormand-Prince step as written (FMA =
# 2; hardware rcp, rsq, sqrt, min, max = 1): six right-hand sides at 84 (of
# which the NFW mass integral 56), five coefficient interpolations at 55,
# stage combinations 184, error norm and step control 182 (the FP64 step
# factor exp/log 77).  A fixed hand count of the method, not a counter
# reading; the hardware counts of the current kernel are in
# profiles/k_dp5_f64_plain_scale.txt.
FLOP_PER_DP5_ATTEMPT = 6 * 84 + 5 * 55 + 184 + 182
FP64_VECTOR_PEAK_TFLOPS = 78.6

# HBM bytes per k_dp5_f64 launch on this workload (1024 threads, 64 workgroups),
# from rocprofv3 FETCH_SIZE and WRITE_SIZE over the five 64-workgroup timed
# launches of an 8-profile run, each scaled by what the counter reads for a
# plain 256 MiB device copy (FETCH x 2.0, WRITE x 0.5).  Valid only for the
# sources and build flags these hashes name; any change to them reports
# traffic as null.
TRAFFIC_BYTES_PER_LAUNCH = 2306784
TRAFFIC_SOURCES = {
    "kernels_f64.hip": "a301c4f141ed72bb07fec410e899b6a8d886a9b29044f427b5ae95a812cc5648",
    "nh_dp5.h": "f549dc045b2dad8c3d0f2295f47c89ee3ccff4ff1b6cb65d38681af7120cf2fd",
    "nh_device.h": "d66562e126b1b11fa0adf9602293e8d61bfae430e550b4280d1c054cb81e9efe",
    "nh_internal.h": "c67215a63146422220ebf4f8d316c7ffef0676c2b6adf91e41aa10bec7ef7786",
    "nh_reduce.h": "0ec2207e398f4b40a854cef770f3d14fc50b1c10969300e7d47dcb95858f54c4",
    "../build.py": "460fa76e681efeee43268db77e28bb7db2f63ba999f4b207719e81dac423d265",
}
METRIC = ("trajectory-steps/s + n/n̄ profiles/s (FP32-comp vs FP64) at ≤1e-4 rel err; p50/p99")


def measured_traffic():
    """Per-launch HBM bytes if the kernel sources are the ones profiled, else None."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2410_08267_amd", "csrc")
    for name, digest in TRAFFIC_SOURCES.items():
        try:
            with open(os.path.join(csrc, name), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return TRAFFIC_BYTES_PER_LAUNCH


def _max_rel(a, b):
    import numpy as np
    return float(np.max(np.abs(np.asarray(a) / np.asarray(b) - 1.0)))


def cpu_baseline_leg(reqs, prof64, prof32, small_req):
    """The oracle (plain C, FP64, one thread per core) on this host, and the GPU's
    profiles against it.

    cpu_baseline: the whole seed-0 profile at the headline's rtol, timed.
    max_rel_err_vs_oracle (max over radii of |n/nbar_gpu / n/nbar_oracle - 1|):
    the FP64 headline's seed-0 profile against that solve (same rtol) and
    against the oracle's reference mode (Dormand-Prince at rtol 1e-10); each
    FP32C profile against the reference mode, seed 0 on every radius, the
    other seeds on every tenth radius.  Also the oracle's time for the small
    case."""
    import numpy as np
    from oracle import oracle as O
    threads = len(os.sched_getaffinity(0))
    res = {}
    req0 = reqs[0]
    t0 = time.perf_counter()
    tr = O.solve(req0, threads=threads)
    dt = time.perf_counter() - t0
    acc, rej = int(tr["accepted"].sum()), int(tr["rejected"].sum())
    res["cpu_baseline"] = {
        "value": acc / dt,
        "unit": "trajectory-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"the whole seed-0 plain-at-scale profile ({req0.n_traj} trajectories, one of the "
                   f"{len(reqs)} timed steps): {acc} accepted + {rej} rejected steps in {dt:.1f} s"),
    }
    print(f"[bench] oracle seed 0 at rtol {req0.rtol:g}: {dt:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ref0 = O.solve(req0.with_(rtol=1e-10), threads=threads)["n_over_nbar"]
    print(f"[bench] oracle seed 0 at rtol 1e-10: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    err = {"seed": 0, "gpu_rtol": req0.rtol}
    if prof64 is not None:
        err["fp64_vs_oracle_same_rtol"] = _max_rel(prof64, tr["n_over_nbar"])
        err["fp64_vs_oracle_reference_rtol_1e-10"] = _max_rel(prof64, ref0)
        err["fp64_per_radius_vs_reference"] = [float(f"{x:.3g}") for x in np.abs(prof64 / ref0 - 1.0)]
    res["max_rel_err_vs_oracle"] = err
    if prof32 is not None:
        per = [_max_rel(prof32[0], ref0)]
        sub = np.arange(0, req0.n_r, 10)
        t0 = time.perf_counter()
        for r, p in zip(reqs[1:], prof32[1:]):
            rq = r.with_(rtol=1e-10, r_kpc=np.asarray(r.r_kpc)[sub])
            per.append(_max_rel(p[sub], O.solve(rq, threads=threads)["n_over_nbar"]))
        print(f"[bench] oracle FP32C checks: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        res["fp32c_max_rel_err_vs_oracle"] = {
            "reference": "oracle Dormand-Prince rtol 1e-10, FP64",
            "per_profile": per,
            "max": max(per),
            "radii": f"seed 0: all {req0.n_r}; seeds 1..{len(reqs) - 1}: every tenth ({sub.size})",
        }
    small = {}
    t0 = time.perf_counter()
    O.solve(small_req, threads=threads)
    small["oracle_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.solve(small_req.with_(method="dp5", rtol=1e-10), threads=threads)
    small["oracle_dp5_rtol1e-10_s"] = time.perf_counter() - t0
    small["oracle_cores"] = threads
    res["small_oracle"] = small
    return res


def batched_leg(ctx, n_req: int, tuned=None):
    """The batched workload (n_req heterogeneous requests, one persistent launch
    each) in FP64 and in the FP32-compensated form: profiles/s of whole batches."""
    import torch
    from paper_2410_08267_amd import workloads as W
    res = {"requests": n_req,
           "workload": ("batched: M0 log-uniform 1e11-1e15 Msun, c0 U[4,15], m U[0.02,0.3] eV, "
                        "N_r U{16..128} x N_y U{32..256} x N_mu U{16..64}, Dormand-Prince rtol 1e-8, z 0->4")}
    for prec in ("fp64", "fp32c"):
        if tuned is not None:
            tuned[f"batch_{prec}"] = tune(ctx, "batch", W.batched(998, n_req=48, prec=prec))
        warm = W.batched(999, n_req=16, prec=prec)
        reqs = W.batched(0, n_req=n_req, prec=prec)
        n_traj = sum(r.n_traj for r in reqs)
        out = torch.empty(sum(r.n_r for r in reqs), dtype=torch.float64, device="cuda")
        ctx.solve_batch(warm, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, _ = ctx.solve_batch(reqs, out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc = sum(st["accepted_steps"] for st in stats)
        att = acc + sum(st["rejected_steps"] for st in stats)
        res[prec] = {
            "profiles_per_s": n_req / dt,
            "seconds": dt,
            "kernel_ms": stats[0]["kernel_ms"],
            "trajectories": n_traj,
            "trajectory_steps_per_s": acc / dt,
            "failed": sum(st["n_failed"] for st in stats),
        }
        if prec == "fp64":
            tf = FLOP_PER_DP5_ATTEMPT * att / (stats[0]["kernel_ms"] / 1e3) / 1e12
            res[prec]["kernel"] = "k_slice_f64"
            res[prec]["achieved_tflops"] = tf
            res[prec]["frac_of_fp64_peak"] = tf / FP64_VECTOR_PEAK_TFLOPS
        print(f"[bench] batched {prec}: {n_req} requests {n_traj} trajectories in {dt:.2f} s", file=sys.stderr,
              flush=True)
    return res


def serving_leg(ctx, capacity: float, prec: str, n_req: int, loads=(0.5, 0.9), warm: int = 50):
    """Poisson arrivals of serving-workload requests at fractions of the batched
    capacity (profiles/s): p50/p99 latency from arrival to result, throughput."""
    import numpy as np
    from paper_2410_08267_amd import nuhalo as N
    from paper_2410_08267_amd import workloads as W
    out = {}
    for frac in loads:
        qps = frac * capacity
        arrivals, reqs = W.serving(17, n_req + warm, qps, prec=prec)
        t0 = time.monotonic()
        pending = {}
        lat = np.full(len(reqs), np.nan)
        done_t = np.full(len(reqs), np.nan)
        i = 0
        while i < len(reqs) or pending:
            now = time.monotonic() - t0
            while i < len(reqs) and arrivals[i] <= now:
                tk = ctx.submit(reqs[i])
                if tk is None:
                    break                     # over budget: retry (latency keeps counting)
                pending[tk] = i
                i += 1
            for tk in list(pending):
                j = pending[tk]
                r = ctx.poll(tk, reqs[j].n_r)
                if r is not None:
                    tdone = time.monotonic() - t0
                    lat[j] = tdone - arrivals[j]
                    done_t[j] = tdone
                    del pending[tk]
            time.sleep(0.0005)
        m = lat[warm:]
        span = np.nanmax(done_t[warm:]) - arrivals[warm]
        # where the tail comes from: latency by quartile of request size
        # (trajectories), smallest first
        size = np.array([r.n_traj for r in reqs[warm:]], dtype=np.float64)
        quart = np.digitize(size, np.quantile(size, [0.25, 0.5, 0.75]))
        by_size = [{"max_trajectories": int(size[quart == b].max()),
                    "p50_ms": float(np.percentile(m[quart == b], 50) * 1e3),
                    "p99_ms": float(np.percentile(m[quart == b], 99) * 1e3)} for b in range(4)]
        out[f"load_{frac:g}"] = {
            "offered_qps": qps,
            "requests": n_req,
            "p50_ms": float(np.percentile(m, 50) * 1e3),
            "p99_ms": float(np.percentile(m, 99) * 1e3),
            "mean_ms": float(np.mean(m) * 1e3),
            "profiles_per_s": n_req / span,
            "by_size_quartile": by_size,
        }
        print(f"[bench] serving {prec} at {frac:g} C: p50 {out[f'load_{frac:g}']['p50_ms']:.1f} ms "
              f"p99 {out[f'load_{frac:g}']['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    return out


def tune(ctx, form: str, reqs):
    """nh_autotune on a sample disjoint from the timed work (untimed)."""
    t0 = time.perf_counter()
    res = ctx.autotune(reqs, form)
    res["seconds"] = time.perf_counter() - t0
    print(f"[bench] autotune {form} {'fp32c' if res['precision'] else 'fp64'}: block {res['block_threads']} "
          f"slots {res['batch_slots']} ({res['best_ms']:.1f} ms vs default {res['default_ms']:.1f} ms)",
          file=sys.stderr, flush=True)
    return res


# Consecutive profiles run side by side on PIPE_DEPTH contexts, each on its own
# stream and its share of the CUs, so that one profile's tail (its few longest
# trajectories) idles only that share.  Each step is still one whole profile.
# Four: one hardware queue each (four per process here); streams beyond that
# share queues and serialise.
PIPE_DEPTH = 4
PLAIN_FP64_BLOCK = 1024   # four waves per SIMD pay once tails no longer idle the device
PLAIN_FP32C_BLOCK = 1024  # four waves per SIMD (the FP32C kernel built for them)
CU_SHARE = 1.0            # workgroups per launch: this many CUs' worth over the profiles in flight


def overlapped(reqs, outs, block, warm_req):
    """Solve reqs[i] into outs[i] on PIPE_DEPTH contexts, each on its own stream
    and capped to its share of the CUs; a context takes the next profile as soon
    as its previous one is done, the profiles taken heaviest halo first.

    Returns the wall time, the summed statistics, each launch's own kernel time,
    the span of GPU work over the timed region from HIP events recorded on every
    stream the kernels run on, the context of the last profile and all contexts."""
    import torch
    from paper_2410_08267_amd import nuhalo as N
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    ctxs = [N.Context(0) for _ in range(PIPE_DEPTH)]
    streams = [torch.cuda.Stream() for _ in range(PIPE_DEPTH)]
    warm_out = torch.empty(warm_req.n_r, dtype=torch.float64, device="cuda")
    for c, s in zip(ctxs, streams):
        if block:
            c.set_option("block_threads", block)
        c.set_option("workgroups", max(1, n_cu // PIPE_DEPTH))
        c.solve_async(warm_req, warm_out, stream=s)
        c.last_stats()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev_end = [None] * PIPE_DEPTH
    tot = {"accepted_steps": 0, "rejected_steps": 0, "fp64_steps": 0}
    kernel_ms = []
    last = None
    t0 = time.perf_counter()
    ev0.record(streams[0])
    for s in streams[1:]:
        s.wait_event(ev0)            # no stream starts before the start event
    # longest expected first: halo mass is the dominant cost driver of a
    # profile (rank correlation 0.91 between M0 and mean attempts per
    # trajectory over the plain-at-scale seeds 0-19, from the oracle), so the
    # heaviest halos start first and the run ends on the cheapest ones
    todo = sorted(zip(reqs, outs), key=lambda ro: -ro[0].M0)
    free = list(range(PIPE_DEPTH))
    busy = {}
    while todo or busy:
        while free and todo:
            k = free.pop(0)
            r, o = todo.pop(0)
            # the last profiles may spread over the CUs the others free as they end
            ctxs[k].set_option("workgroups", max(1, int(CU_SHARE * n_cu) // max(1, min(PIPE_DEPTH, len(todo) + 1))))
            ctxs[k].solve_async(r, o, stream=streams[k])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(streams[k])
            ev_end[k] = ev
            busy[k] = ev
            last = ctxs[k]
        done = [k for k, ev in busy.items() if ev.query()]
        if not done:
            time.sleep(2e-5)
            continue
        for k in done:
            st, _ = ctxs[k].last_stats()
            for key in tot:
                tot[key] += st[key]
            kernel_ms.append(st["kernel_ms"])
            del busy[k]
            free.append(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    span_ms = max(ev0.elapsed_time(e) for e in ev_end if e is not None)
    return wall, tot, kernel_ms, span_ms, last, ctxs


def plain_leg(ctx, stream, reqs, warmup, tuned=None):
    """The headline: one FP64 profile of the plain-at-scale workload per step."""
    import torch
    from paper_2410_08267_amd import workloads as W
    block = PLAIN_FP64_BLOCK
    if tuned is not None:
        tuned["plain_fp64"] = tune(ctx, "plain", [W.plain_scale(s) for s in (2000, 2001, 2002)])
        block = tuned["plain_fp64"]["block_threads"]
    out = torch.empty(128, dtype=torch.float64, device="cuda")
    for i in range(warmup):
        ctx.solve_async(W.plain_scale(1000 + i), out, stream=stream)
        ctx.last_stats()
    outs = [torch.empty(r.n_r, dtype=torch.float64, device="cuda") for r in reqs]
    dt, tot, kernel_ms, span_ms, last, ctxs = overlapped(reqs, outs, block, W.plain_scale(1000))
    acc, rej = tot["accepted_steps"], tot["rejected_steps"]
    for c in ctxs:
        c.close()
    profiles = [o.cpu().numpy() for o in outs]
    # step-count structure of the last timed profile, from a solve that keeps
    # per-trajectory results (outside the timed region; same bits)
    r = reqs[-1]
    ctx.set_option("trajectory_stats", 1)
    ctx.solve_async(r, torch.empty(r.n_r, dtype=torch.float64, device="cuda"), stream=stream)
    ctx.last_stats()
    acc_t, rej_t, _ = ctx.trajectory_stats(r.n_traj)
    ctx.set_option("trajectory_stats", 0)
    att = (acc_t.astype("int64") + rej_t).reshape(r.n_r, r.n_y, r.n_mu)
    import numpy as np
    blocks = lambda a, axis, n: [float(x.mean()) for x in np.array_split(np.moveaxis(a, axis, 0), n)]
    steps_hist = {
        "seed": len(reqs) - 1,
        "attempts_percentiles": {q: float(np.percentile(att, float(q))) for q in ("50", "90", "99", "99.9", "100")},
        "mean_attempts_by_radius_decile": blocks(att, 0, 10),
        "mean_attempts_by_momentum_decile": blocks(att, 1, 10),
        "mean_attempts_by_direction_decile": blocks(att, 2, 10),
    }
    # launches overlap, so the kernel's time per profile is the span of GPU work
    # over the timed region (HIP events on every stream) divided by the profiles
    span_per_profile = span_ms / len(reqs)
    achieved = FLOP_PER_DP5_ATTEMPT * (acc + rej) / (span_ms / 1e3) / 1e12
    return profiles, {
        "value": acc / dt,
        "ms_per_step": dt / len(reqs) * 1e3,
        "profiles_per_s": len(reqs) / dt,
        "accepted_steps": acc,
        "rejected_steps": rej,
        "kernel_ms_per_profile": span_per_profile,
        "kernel_ms_avg": sum(kernel_ms) / len(kernel_ms),
        "concurrent_profiles": PIPE_DEPTH,
        "steps_per_trajectory": steps_hist,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            # measured for the default launch shape only
            "traffic": measured_traffic() if block == PLAIN_FP64_BLOCK else None,
            "traffic_unit": "bytes per launch",
            "kernel": "k_dp5_f64",
            "flop_per_attempt": FLOP_PER_DP5_ATTEMPT,
            "time_basis": "span of GPU work over the timed profiles / profiles (launches overlap)",
        },
    }


def small_leg(ctx, stream):
    """The small plain case (10 x 50 x 20 trajectories, RK4 with 1000 fixed steps):
    157 waves for 1024 SIMDs, so latency-bound on the GPU; reported, not gated.
    Also the same case with Dormand-Prince at rtol 1e-10.  (The oracle's time
    for both: the cpu_baseline leg.)"""
    import torch
    from paper_2410_08267_amd import workloads as W
    req = W.plain_small()
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out, stream=stream)
    ctx.last_stats()
    ms = []
    for _ in range(5):
        t0 = time.perf_counter()
        ctx.solve_async(req, out, stream=stream)
        st, _ = ctx.last_stats()
        ms.append((time.perf_counter() - t0) * 1e3)
    res = {"workload": "plain_small: 10 r x 50 y x 20 mu, RK4 1000 steps, z 0->4",
           "trajectories": req.n_traj, "steps": st["accepted_steps"],
           "gpu_ms": min(ms), "gpu_kernel_ms": st["kernel_ms"],
           "gpu_trajectory_steps_per_s": st["accepted_steps"] / (min(ms) / 1e3)}
    # the same case with Dormand-Prince at rtol 1e-10 (the oracle's reference mode)
    ref = req.with_(method="dp5", rtol=1e-10)
    ctx.solve_async(ref, out, stream=stream)
    ctx.last_stats()
    t0 = time.perf_counter()
    ctx.solve_async(ref, out, stream=stream)
    st2, _ = ctx.last_stats()
    res["gpu_dp5_rtol1e-10_ms"] = (time.perf_counter() - t0) * 1e3
    res["dp5_rtol1e-10_steps"] = st2["accepted_steps"]
    return req, res


def fp32c_leg(ctx, stream, reqs, prof64=None, tuned=None):
    """The FP32-compensated form on the same halos: profiles/s and deviation from
    the FP64 path's profiles (prof64; solved here when not given)."""
    import numpy as np
    import torch
    from paper_2410_08267_amd import workloads as W
    if prof64 is None:
        out = torch.empty(128, dtype=torch.float64, device="cuda")
        prof64 = []
        for r in reqs:
            ctx.solve_async(r, out, stream=stream)
            ctx.last_stats()
            prof64.append(out[:r.n_r].cpu().numpy().copy())
    reqs32 = [r.with_(precision="fp32c") for r in reqs]
    if tuned is not None:
        tuned["plain_fp32c"] = tune(ctx, "plain", [W.plain_scale(s).with_(precision="fp32c")
                                                   for s in (2000, 2001, 2002)])
    outs = [torch.empty(r.n_r, dtype=torch.float64, device="cuda") for r in reqs32]
    block = tuned["plain_fp32c"]["block_threads"] if tuned else PLAIN_FP32C_BLOCK
    dt32, tot, _, span_ms, _, ctxs = overlapped(reqs32, outs, block,
                                                W.plain_scale(1000).with_(precision="fp32c"))
    for c in ctxs:
        c.close()
    acc32, rej32, f64 = tot["accepted_steps"], tot["rejected_steps"], tot["fp64_steps"]
    profiles = [o.cpu().numpy() for o in outs]
    errs = [float(np.max(np.abs(p / p64 - 1.0))) for p, p64 in zip(profiles, prof64)]
    achieved = FLOP_PER_DP5_ATTEMPT * (acc32 + rej32) / (span_ms / 1e3) / 1e12
    return profiles, {
        "trajectory_steps_per_s": acc32 / dt32,
        "profiles_per_s": len(reqs32) / dt32,
        "ms_per_step": dt32 / len(reqs32) * 1e3,
        "concurrent_profiles": PIPE_DEPTH,
        "fp64_attempts": f64,
        "max_rel_err_vs_fp64_path": max(errs),
        "rtol": reqs32[0].rtol,
        "rtol_floor": 1e-7,
        # the same algorithmic FLOP per attempted step, mostly in FP32; packed
        # FP32 math (the datasheet's 157.3) is compiled out, so non-packed FP32
        # issues at the FP64 rate, 78.6, the peak the fraction is taken against
        "roofline": {"bound": "alu", "kernel": "k_dp5_f32c", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "peak_packed_fp32": 157.3, "unit": "TFLOP/s"},
    }


def next_leg(ctx, stream):
    """The rows beyond the headline path, timed on full-size requests of the
    headline's shape (100 r x 200 y x 64 mu, rtol 1e-8, FP64), one profile at a
    time on the whole device:
      masses    - several relic masses from one integration (Sec. II.D), against
                  plain solves at the same velocities (y scaled by m_k/m);
      cull_exit - the App. B cull with the exact free-streaming exit, on and off,
                  on the lightest halo of the headline's seeds (its outer radii
                  lie beyond the compensation radius); the profiles must be the
                  same bits;
      variants  - the Sec. IV halo variants (growth xi^alpha, early onset, the
                  G modulations kappa_1 and kappa_2) and observation at z0 > 0;
      integrand - the profile plus the relic distribution behind it (Fig. 3),
                  against the plain solve of the same request.
    Their parity with the oracle is covered by the GPU tests at reduced sizes."""
    import numpy as np
    import torch
    from paper_2410_08267_amd import workloads as W

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def rate(st):
        att = st["accepted_steps"] + st["rejected_steps"]
        tf = FLOP_PER_DP5_ATTEMPT * att / (st["kernel_ms"] / 1e3) / 1e12
        return {"kernel_ms": st["kernel_ms"], "attempted_steps": att, "achieved_tflops": tf,
                "frac": tf / FP64_VECTOR_PEAK_TFLOPS}

    def one(req):
        out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
        dt = timed(lambda: ctx.solve_async(req, out, stream=stream))
        st, _ = ctx.last_stats()
        return out.cpu().numpy(), st, dt

    def rel(a, b):
        return float(np.max(np.abs(np.asarray(a) / np.asarray(b) - 1.0)))

    one(W.plain_scale(1000))
    res = {}

    req = W.plain_scale(0)
    masses = [float(m) for m in np.geomspace(0.02, 0.3, 8)]
    out = torch.empty(len(masses) * req.n_r, dtype=torch.float64, device="cuda")
    ctx.solve_masses(req, masses, out, stream=stream)
    ctx.last_stats()
    dt_m = timed(lambda: ctx.solve_masses(req, masses, out, stream=stream))
    st_m, _ = ctx.last_stats()
    pm = out.cpu().numpy().reshape(len(masses), req.n_r)
    dt_p, err = 0.0, 0.0
    for i, mk in enumerate(masses):
        p, _, dt = one(req.with_(m_eV=mk, y=req.y * (mk / req.m_eV)))
        dt_p += dt
        err = max(err, rel(pm[i], p))
    res["masses"] = {"request": f"plain_scale seed 0 (m = {req.m_eV} eV), masses {masses[0]:.3g}-{masses[-1]:.3g} eV",
                     "masses": len(masses), "seconds": dt_m, "profiles_per_s": len(masses) / dt_m,
                     "plain_seconds": dt_p, "speedup_vs_plain": dt_p / dt_m,
                     "max_rel_diff_vs_plain": err, **rate(st_m)}

    seeds = {s: W.plain_scale(s) for s in range(16)}
    s_light = min(seeds, key=lambda s: seeds[s].M0)
    light = seeds[s_light]
    p_on, st_on, dt_on = one(light)
    ctx.set_option("free_exit", 0)
    try:
        p_off, st_off, dt_off = one(light)
    finally:
        ctx.set_option("free_exit", 1)
    res["cull_exit"] = {"request": f"plain_scale seed {s_light} (M0 = {light.M0:.3g} Msun)",
                        "seconds_on": dt_on, "seconds_off": dt_off, "speedup": dt_off / dt_on,
                        "same_bits": bool(np.array_equal(p_on, p_off)),
                        "free_exits": st_on["free_exits"],
                        "attempted_steps_on": st_on["accepted_steps"] + st_on["rejected_steps"],
                        "attempted_steps_off": st_off["accepted_steps"] + st_off["rejected_steps"]}

    base = W.plain_scale(0).with_(mass_kind="paper", M0=1.0e14, conc_kind="constant", c0=7.0)
    variants = {"paper_halo": base, "xi_alpha_0.5": base.with_(mass_alpha=0.5),
                "xi_alpha_2": base.with_(mass_alpha=2.0), "early_onset_z9": base.with_(z_form=9.0),
                "kappa_1": base.with_(kappa_kind="paper", kappa_a=0.2, kappa_b=1.5),
                "kappa_2": base.with_(kappa_kind="paper", kappa_a=0.1, kappa_b=0.8),
                "z_obs_0.5": base.with_(z_obs=0.5)}
    res["variants"] = {"request": "plain_scale seed 0 grids, the paper's halo with M_h = 1e14 Msun, c = 7"}
    for name, r in variants.items():
        _, st, dt = one(r)
        res["variants"][name] = {"seconds": dt, **rate(st)}

    p, st_p, dt_p = one(req)
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    integ = torch.empty(req.n_r * req.n_y, dtype=torch.float64, device="cuda")
    dt_i = timed(lambda: ctx.solve_integrand(req, out, integ, stream=stream))
    st_i, _ = ctx.last_stats()
    res["integrand"] = {"request": "plain_scale seed 0", "seconds": dt_i, "plain_seconds": dt_p,
                        "same_profile_bits": bool(np.array_equal(out.cpu().numpy(), p)), **rate(st_i)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="plain,fp32c,batched,serving,next",
                    help="comma list of legs: plain (the headline value), fp32c, batched, serving, "
                         "next (multi-mass reuse, cull, halo variants, integrand output)")
    ap.add_argument("--no-fp32c", dest="fp32c", action="store_false",
                    help="skip the FP32-compensated leg")
    ap.add_argument("--no-batched", dest="batched", action="store_false",
                    help="skip the batched leg (heterogeneous requests in one launch)")
    ap.add_argument("--batch-requests", type=int, default=512)
    ap.add_argument("--no-serving", dest="serving", action="store_false",
                    help="skip the serving leg (Poisson arrivals, p50/p99 latency)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--tune", action="store_true",
                    help="run nh_autotune first (untimed, on samples disjoint from the timed work); "
                         "the built-in launch shapes are the ones it picked on MI355X")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (counter calibration)")
    args = ap.parse_args()
    legs = set(args.legs.split(","))
    args.fp32c = args.fp32c and "fp32c" in legs
    args.batched = args.batched and "batched" in legs
    args.serving = args.serving and "serving" in legs
    plain = "plain" in legs

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the profile path is built and measured on a single "
              "MI355X (trajectories shard by radius across GPUs with no exchange; not built here).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2410_08267_amd import nuhalo as N
    from paper_2410_08267_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        # a plain device-to-device copy of known size: reads and writes BYTES once
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}), flush=True)
        return
    ctx = N.Context(0)
    stream = torch.cuda.current_stream(dev)
    reqs = [W.plain_scale(s) for s in range(args.steps)]
    line = {
        "metric": METRIC,
        "value": None,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("plain_scale: one NFW halo per step (M0 log-uniform 1e11-1e15 Msun, c0 U[4,15], "
                         "m in {0.05,0.1,0.3} eV), 100 r x 200 y x 64 mu = 1.28M trajectories, "
                         "Dormand-Prince 5(4) rtol 1e-8, FP64, z 0->4, seeds 0..K-1"),
            "trajectories_per_step": reqs[0].n_traj,
            "precision": "fp64",
        },
        # context, not a target: the paper (abstract, Sec. V) reports that its
        # method gives a profile in a matter of seconds, on hardware it does not name
        "paper_context": "a profile in seconds (abstract, Sec. V); the paper's hardware is not stated",
    }
    tuned = {} if args.tune else None
    prof64 = prof32 = None
    if plain:
        prof64, res = plain_leg(ctx, stream, reqs, args.warmup, tuned)
        line.update(res)
        measured = ctx.fp64_fma_peak()
        line["roofline"]["peak_measured"] = measured
        line["roofline"]["frac_of_measured_peak"] = line["roofline"]["achieved"] / measured
        # threads per workgroup of the plain FP64 kernel (one workgroup per CU,
        # a quarter of the CUs per profile): the bench's choice or the autotuner's
        blk = tuned["plain_fp64"]["block_threads"] if tuned else PLAIN_FP64_BLOCK
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        line["occupancy"] = {"threads_per_workgroup": blk, "waves_per_simd": blk / 256,
                             "workgroups_per_launch": max(1, n_cu // PIPE_DEPTH),
                             "concurrent_profiles": PIPE_DEPTH,
                             "lds_table_bytes_per_cu": 3073 * 5 * 8}
    small_req = None
    if plain:
        small_req, line["small"] = small_leg(ctx, stream)
    if args.fp32c:
        prof32, line["fp32c"] = fp32c_leg(ctx, stream, reqs, prof64, tuned)
    if args.batched:
        line["batched"] = batched_leg(ctx, args.batch_requests, tuned)
    if "next" in legs:
        line["next_rows"] = next_leg(ctx, stream)
    if args.serving and args.batched:
        serving = {}
        for pr in ("fp32c", "fp64"):
            cap = line["batched"][pr]["profiles_per_s"]
            serving[pr] = serving_leg(ctx, cap, pr, args.serve_requests)
            serving[pr]["capacity_profiles_per_s"] = cap
        line["serving"] = serving
    if tuned:
        line["tuned"] = tuned
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(reqs, prof64[0] if prof64 else None, prof32, small_req or W.plain_small())
        line["cpu_baseline"] = cpu["cpu_baseline"]
        line["max_rel_err_vs_oracle"] = cpu["max_rel_err_vs_oracle"]
        if "fp32c" in line and "fp32c_max_rel_err_vs_oracle" in cpu:
            line["fp32c"]["max_rel_err_vs_oracle"] = cpu["fp32c_max_rel_err_vs_oracle"]
        if "small" in line:
            line["small"].update(cpu["small_oracle"])
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
