#!/usr/bin/env python3
"""Benchmark of the MOL^T Cahn-Hilliard hot path on one MI355X.

Workload (default): 2D Cahn-Hilliard, 4096 x 4096 periodic nodes on [0,1]^2,
eps = 0.005, BDF2 (BE start-up step), dt = 1e-5, fixed-point tolerance 1e-8,
quadrature order M = 4, FP32 sweeps (FP64 weights, boundary solves, residual,
mass and energy), u0 = 0.3 + 0.05 N(0,1) from the seeded generator.  One
benchmark step is one ch_step (the whole hot path: rhs, R = A1^-1 A2^-1 rhs,
the fixed-point iterations to tolerance, the final update and reductions) on
device-resident fields.  W warm-up steps run first (the BE start-up step and
the first BDF2 steps), then K timed steps.

Metric: Gpt-sweeps/s = executed point-sweeps / s, one point-sweep being one 1D
inverse applied to one grid point: 4 per point per step for R plus 7 per point
per fixed-point iteration (the passes P1..P4 apply 2+2+2+1 line inverses).  The
nominal count of the method (8 per iteration) and the point-iteration rate are
reported beside it.

Also printed on the same JSON line:
  roofline      the dominant kernel's algorithmic HBM bytes per launch divided
                by its average duration, timed with HIP events on the library's
                launch stream over the timed region, against 8 TB/s (the last
                warm-up step times every kernel, which names the dominant one
                and gives the `kernels` breakdown; the timed steps time that
                kernel alone, as events around every launch slow the stream);
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload
                (first BE step of the full field with a fixed number of
                iterations), on this host's cores;
  batched       the batched workload (256 seeded instances of uneven sizes and
                parameters, shapes autotuned): ch_solve_batch against one plain
                ch_solve per instance, steps/s and Gpt-sweeps/s of each;
  served        the served workload (Poisson arrivals of vector-model
                requests): continuous batching against a plain FIFO of
                ch_solve calls, p50/p99 latency and steps/s of each, also at a
                sub-capacity rate and near capacity;
  error         the FP32 result's max-abs and L2 error: against the FP64 path
                on the full field (two steps), and against the FP64 oracle on a
                periodic patch with the workload's grid spacing, eps and dt;
  sweep         the standalone line inverse (mol_t_helmholtz_sweep) along x
                and along y of the 4096^2 field, FP32 and FP64: Gpt-sweeps/s and
                the fraction of 8 TB/s;
  full_workload the whole 500-step workload once from u0: per-step iteration
                counts (first, last, range), wall time and rates, and the FP32
                result's error against the same steps in FP64;
  ch1d, ch2d_neumann  the 1D (N=256, BE, FP64, 200 steps) and 512^2 Neumann
                (BDF2, 2000 steps, FP64 then FP32) workloads: steps/s on the
                GPU and of the oracle (one core and all cores), errors.
The process frees its device memory and prints the JSON line last.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per grid point of one launch of the FP32 iteration
# kernels (increment form: every FP32 iteration after a step's FP64 first one):
# field reads + writes; the single-read y-pass (timed under the yfin kinds)
# also writes its per-segment totals, the combine reads them and writes the
# seeds, and the next x-pass reads the seeds (2 fields x 2 directions x 4 B per
# 64-row segment: 0.25 B per point each).
BYTES_PER_POINT = {
    "yfin_P1": 12 + 8 + 0.25,
    "ycomb_P1": 0.5,
    "xpass_P2": 20 + 8 + 0.25,
    "yfin_P3": 8 + 8 + 0.25,
    "ycomb_P3": 0.5,
    "xpass_P4": 16 + 8 + 0.25,
}
# one whole FP32 iteration with every field read once and written once:
# P1 3 reads + 2 writes, P2 5 + 2, P3 2 + 2, P4 4 + 2, 4 B each
ITER_BYTES_PER_POINT = 88.0


COUNTERS = os.path.join(ROOT, "profiles", "linepass_4096_fp32_hbm_counters.md")
# what decides the x-pass kernel's code: its sources and the compile flags
KERNEL_SOURCES = ("csrc/molt_device.h", "csrc/molt_kernels.hip", "csrc/molt_internal.h", "build.py")


def counter_traffic(kernel: str, n: int):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (calibrated FETCH_SIZE + WRITE_SIZE), or None when the summary is for
    another kernel or size, or the kernel sources changed since it was taken."""
    import hashlib
    if n != 4096 or not os.path.exists(COUNTERS):
        return None
    kv = {}
    for line in open(COUNTERS):
        if "=" in line and line.startswith("    "):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_04214_amd", f), "rb") as fh:
            h.update(fh.read())
    if kv.get("kernel") != kernel or kv.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed time steps")
    ap.add_argument("--warmup", type=int, default=2, help="untimed time steps before the timed ones")
    ap.add_argument("--n", type=int, default=4096, help="grid side (default: the 4096^2 workload)")
    ap.add_argument("--init", choices=["prev", "linear"], default="linear")
    ap.add_argument("--max-iter", type=int, default=50000, help="iteration cap per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=24, help="oracle iterations in the CPU sample")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="steps per instance of the batched workload (0: skip it)")
    ap.add_argument("--batch-count", type=int, default=256, help="instances of the batched workload")
    ap.add_argument("--no-batch-plain", action="store_true", help="skip the plain-path timing of the batch")
    ap.add_argument("--serve-count", type=int, default=200,
                    help="requests of the served workload (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrival rate of the served workload (1/s)")
    ap.add_argument("--serve-sub-count", type=int, default=200,
                    help="requests of the sub-capacity and near-capacity served traces (0: skip them)")
    ap.add_argument("--no-small", action="store_true", help="skip the 1D and 512^2 Neumann workloads")
    ap.add_argument("--full-steps", type=int, default=500,
                    help="steps of the whole-workload run (the workload's 500; 0: skip it)")
    ap.add_argument("--no-full-fp64", dest="full_fp64", action="store_false",
                    help="skip the FP64 run of the whole workload (its FP32 error)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the standalone sweep measurement")
    ap.add_argument("--no-error", action="store_true", help="skip the FP32 error measurement")
    ap.add_argument("--c2-steps", type=int, default=2000, help="steps of the 512^2 Neumann workload")
    ap.add_argument("--no-profile", action="store_true", help="do not time kernels with HIP events")
    ap.add_argument("--shape", type=str, default="auto",
                    help="line-block shape of the workload's line length: 'auto' (autotuned), 'default' "
                         "(the library's table) or 'kx,ky'")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                      "launches": 3}))


def run_batched(args, molt, synth):
    """The batched workload: `count` seeded instances (sides 64..1024
    log-uniform, eps, dt, boundary and stepper drawn per instance, FP32, tol
    1e-8), line-block shapes autotuned first; ch_solve_batch against one plain
    ch_solve per instance on the same GPU and the same inputs."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    table = molt.autotune(molt.MOLT_F32, 1024)
    tune_s = time.perf_counter() - t0
    inst = synth.batch_instances(args.batch_count, steps=args.batch_steps)

    def spec(d):
        bc = molt.MOLT_BC_PERIODIC if d["bc"] == "periodic" else molt.MOLT_BC_NEUMANN
        g = molt.make_grid(d["n"], d["n"], 0.0, d["L"], 0.0, d["L"], bc, d["M"])
        p = molt.make_params(d["eps"], d["dt"], tol=d["tol"], max_iter=20000, init=molt.MOLT_INIT_LINEAR,
                             stepper=molt.MOLT_BDF2 if d["stepper"] == "BDF2" else molt.MOLT_BE,
                             precision=molt.MOLT_F32)
        return g, p

    u0 = [torch.tensor(synth.instance_u0(d), dtype=torch.float32, device="cuda:0") for d in inst]
    xs = [u.clone() for u in u0]
    specs = [spec(d) + (xs[i], args.batch_steps) for i, d in enumerate(inst)]
    work = molt.workspace(molt.ch_batch_workspace_bytes(molt.make_instances(specs), len(specs)))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        t0 = time.perf_counter()
        st, recs = molt.solve_batch(specs, work=work)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    iters = [[r.iters for r in rr] for rr in recs]
    pts = np.array([d["n"] ** 2 for d in inst], dtype=np.float64)
    sweeps = float(sum(pts[i] * sum(4 + 7 * k for k in iters[i]) for i in range(len(inst))))
    nsteps = args.batch_steps * len(inst)
    ticks = [sum(1 + k for k in it) for it in iters]
    out = {"workload": f"{len(inst)} instances, sides 64..1024 log-uniform (sum n^2 = {int(pts.sum())}), "
                       f"eps U[0.005,0.05], dt U[1e-6,1e-4], periodic/Neumann, BE/BDF2, FP32 tol 1e-8, "
                       f"{args.batch_steps} steps each, u0 = 0.05 U(-1,1)",
           "status": st, "batched_s": round(tb, 3), "batched_steps_per_s": round(nsteps / tb, 1),
           "batched_gpt_sweeps_per_s": round(sweeps / tb / 1e9, 2),
           "ticks_max": max(ticks), "ticks_median": int(np.median(ticks)),
           "us_per_tick_upper_bound_longest": round(1e6 * tb / max(ticks), 1),
           "mean_iters_per_step": round(float(np.mean([np.mean(x) for x in iters])), 1),
           "autotune_s": round(tune_s, 3), "shape_table_fp32": table[:4]}
    if not args.no_batch_plain:
        xp = [u.clone() for u in u0]
        ws = molt.workspace(max(molt.ch_workspace_bytes(*spec(d)) for d in inst))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters_p, secs_p = [], []
        for i, d in enumerate(inst):
            g, p = spec(d)
            ti = time.perf_counter()
            _, infos = molt.solve(xp[i], g, p, args.batch_steps, work=ws)
            secs_p.append(time.perf_counter() - ti)
            iters_p.append([r.iters for r in infos])
            if (i + 1) % 32 == 0:
                print(f"batched: plain path {i + 1}/{len(inst)} instances, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out.update({"plain_s": round(tp, 3), "plain_steps_per_s": round(nsteps / tp, 1),
                    "speedup_vs_plain": round(tp / tb, 2),
                    "bitwise_equal_to_plain": all(torch.equal(xp[i], xs[i]) for i in range(len(inst))),
                    "same_iterations_as_plain": iters_p == iters})
        # the instance with the most ticks sets the batch's wall time: alone
        # in a batch of one and on the plain path
        k = int(np.argmax(ticks))
        d = inst[k]
        xt = u0[k].clone()
        g, p = spec(d)
        with torch.cuda.stream(s):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            molt.solve_batch([(g, p, xt, args.batch_steps)])
            torch.cuda.synchronize()
            ta = time.perf_counter() - t0
        out["tail"] = {"instance": k, "n": d["n"], "bc": d["bc"], "stepper": d["stepper"], "ticks": ticks[k],
                       "iters_per_step_mean": round(float(np.mean(iters[k])), 1),
                       "alone_in_a_batch_s": round(ta, 3), "us_per_tick_alone": round(1e6 * ta / ticks[k], 1),
                       "plain_s": round(secs_p[k], 3),
                       "us_per_iteration_plain": round(1e6 * secs_p[k] / max(sum(iters[k]), 1), 1),
                       "alone_share_of_batched_s": round(ta / tb, 3),
                       "bitwise_equal_to_batched": bool(torch.equal(xt, xs[k]))}
    print(f"batched: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def _serve_spec(molt, d):
    bc = molt.MOLT_BC_PERIODIC if d["bc"] == "periodic" else molt.MOLT_BC_NEUMANN
    g = molt.make_grid(d["n"], d["n"], 0.0, d["L"], 0.0, d["L"], bc, d["M"])
    p = molt.make_params(d["eps"], d["dt"], tol=d["tol"], max_iter=20000, init=molt.MOLT_INIT_LINEAR,
                         stepper=molt.MOLT_BDF2 if d["stepper"] == "BDF2" else molt.MOLT_BE,
                         precision=molt.MOLT_F32, model=molt.MOLT_MODEL_VCH)
    return g, p


def _serve_trace(molt, reqs, u0, arrivals, pool_bytes):
    """Real-time serving of a trace: requests are submitted when the wall clock
    passes their arrival time; returns (latencies, makespan, fields)."""
    import numpy as np
    import torch
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    done, fields = {}, {}
    with torch.cuda.stream(s):
        srv = molt.Server(molt.MOLT_F32, 128, pool_bytes)
        t0 = time.perf_counter()
        k = 0
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while k < len(reqs) and arrivals[k] <= now:
                g, p = _serve_spec(molt, reqs[k])
                fields[k] = torch.from_numpy(u0[k]).to("cuda:0")
                srv.submit(g, p, fields[k], reqs[k]["steps"], k)
                k += 1
            active, queued = srv.run(1)
            for r in srv.poll():
                done[r.id] = time.perf_counter() - t0
                if len(done) % 25 == 0:
                    print(f"served trace: {len(done)}/{len(reqs)} done at {done[r.id]:.1f} s", file=sys.stderr,
                          flush=True)
            if active == 0 and queued == 0 and k < len(reqs):
                time.sleep(max(0.0, arrivals[k] - (time.perf_counter() - t0)))
        srv.close()
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    lat = np.array([done[i] - arrivals[i] for i in range(len(reqs))])
    return lat, makespan, fields


def run_served(args, molt, synth):
    """The served workload: Poisson arrivals of vector-model requests (sides
    128..2048 log-uniform, 10..500 steps), served by continuous batching
    (molt_server_*) in real time, against a plain FIFO that solves one request
    at a time with ch_solve on the same GPU (its latencies follow from the
    measured solve times: start = max(arrival, previous finish)).  Then a
    sub-capacity trace: the first requests at half the measured served rate."""
    import numpy as np
    import torch
    reqs = synth.serve_requests(args.serve_count, args.serve_rate)
    u0 = [synth.u0_vch(d["seed"], d["n"], d["n"], d["stream"]).astype(np.float32) for d in reqs]
    arrivals = [d["arrival"] for d in reqs]
    free, _ = torch.cuda.mem_get_info()
    pool = int(min(64 << 30, free // 2))
    lat, makespan, fields = _serve_trace(molt, reqs, u0, arrivals, pool)
    steps = sum(d["steps"] for d in reqs)
    # plain FIFO: measured solve times, queueing from the arrival times
    durs, same = [], True
    for i, d in enumerate(reqs):
        g, p = _serve_spec(molt, d)
        x = torch.from_numpy(u0[i]).to("cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        molt.solve(x, g, p, d["steps"])
        torch.cuda.synchronize()
        durs.append(time.perf_counter() - t0)
        same = same and torch.equal(x.cpu(), fields[i].cpu())
        if (i + 1) % 25 == 0:
            print(f"plain FIFO: {i + 1}/{len(reqs)} solved, busy {sum(durs):.1f} s", file=sys.stderr, flush=True)

    def fifo(arr, dur):
        fin, out = 0.0, []
        for a, du in zip(arr, dur):
            fin = max(a, fin) + du
            out.append(fin - a)
        return np.array(out), fin - arr[0]

    flat, fspan = fifo(arrivals, durs)
    pct = lambda a, q: round(float(np.percentile(a, q)), 4)
    out = {"workload": f"{len(reqs)} vector-model requests (three-phase VCH, sigma0 18), Poisson arrivals at "
                       f"{args.serve_rate}/s, sides 128..2048 log-uniform, 10..500 steps, eps U[0.005,0.05], "
                       f"dt U[1e-6,1e-4], periodic/Neumann, BE/BDF2, FP32 tol 1e-8",
           "requests": len(reqs), "total_steps": steps, "pool_bytes": pool,
           "served": {"p50_s": pct(lat, 50), "p99_s": pct(lat, 99), "makespan_s": round(makespan, 3),
                      "steps_per_s": round(steps / makespan, 1)},
           "fifo_plain": {"p50_s": pct(flat, 50), "p99_s": pct(flat, 99), "makespan_s": round(fspan, 3),
                          "steps_per_s": round(steps / fspan, 1), "busy_s": round(sum(durs), 3)},
           "bitwise_equal_to_plain": same}
    if args.serve_sub_count > 0:
        # the same requests re-timed at half and at 0.9 of the measured served
        # throughput (the overloaded trace's requests per second)
        m = min(args.serve_sub_count, len(reqs))
        cap = len(reqs) / makespan
        out["capacity_req_per_s"] = round(cap, 3)
        for key, frac in (("sub_capacity", 0.5), ("near_capacity", 0.9)):
            rate = frac * cap
            sub_arr = [arrivals[i] * args.serve_rate / rate for i in range(m)]
            slat, sspan, _ = _serve_trace(molt, reqs[:m], u0[:m], sub_arr, pool)
            sflat, _ = fifo(sub_arr, durs[:m])
            out[key] = {"rate_per_s": round(rate, 3), "requests": m,
                        "served": {"p50_s": pct(slat, 50), "p99_s": pct(slat, 99), "makespan_s": round(sspan, 3)},
                        "fifo_plain": {"p50_s": pct(sflat, 50), "p99_s": pct(sflat, 99)}}
    print(f"served: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def host_threads() -> int:
    """Threads for the oracle's all-core leg: OMP_NUM_THREADS when set (the
    process's share of the host), else the logical CPUs."""
    try:
        return max(1, int(os.environ["OMP_NUM_THREADS"]))
    except (KeyError, ValueError):
        return os.cpu_count() or 1


def cpu_info():
    """(model name, logical CPUs) of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def run_error(molt, synth, oracle, w, n):
    """Max-abs and L2 error of the FP32 path on the 4096^2 workload: two steps
    (BE start-up, one BDF2 step) of the full field in FP32 and in FP64 on the
    GPU (the FP64 path matches the oracle to 1e-12 relative in the tests), and
    three steps of a 256^2 periodic patch with the workload's grid spacing,
    eps and dt against the FP64 oracle at the same tolerance."""
    import numpy as np
    import torch
    out = {}
    grid = molt.make_grid(n, n, 0.0, w["L"], 0.0, w["L"], molt.MOLT_BC_PERIODIC, w["M"])
    u0 = synth.workload_u0("ch2d_periodic_bdf2_4096", n)
    res = {}
    for prec, dt in ((molt.MOLT_F64, torch.float64), (molt.MOLT_F32, torch.float32)):
        p = molt.make_params(w["eps"], w["dt"], tol=w["tol"], stepper=molt.MOLT_BDF2, max_iter=20000,
                             init=molt.MOLT_INIT_LINEAR, precision=prec)
        x = torch.tensor(u0, dtype=dt, device="cuda:0")
        (st, infos), _ = _timed(lambda: molt.solve(x, grid, p, 2))
        res[prec] = (x.double().cpu().numpy(), [i.iters for i in infos], infos[-1].mass)
        del x
    d = res[molt.MOLT_F32][0] - res[molt.MOLT_F64][0]
    out["full_field_vs_fp64_gpu"] = {
        "steps": 2, "max_abs": float(np.abs(d).max()), "l2": float(np.sqrt((d ** 2).mean())),
        "iters_fp32": res[molt.MOLT_F32][1], "iters_fp64": res[molt.MOLT_F64][1],
        "mass_fp32_minus_fp64": res[molt.MOLT_F32][2] - res[molt.MOLT_F64][2]}
    m = 256
    L = w["L"] * m / n
    g = molt.make_grid(m, m, 0.0, L, 0.0, L, molt.MOLT_BC_PERIODIC, w["M"])
    up = synth.u0_normal_noise(synth.BASE_SEED + 7, m, m, 0.3, 0.05)
    og = oracle.Grid(nx=m, ny=m, x0=0.0, x1=L, y0=0.0, y1=L, bc=oracle.BC_PERIODIC, M=w["M"])
    po = oracle.Params(eps=w["eps"], dt=w["dt"], tol=w["tol"], stepper=oracle.BDF2, max_iter=20000,
                       init=oracle.INIT_LINEAR)
    ref, rinf = oracle.solve(og, po, up, 3)
    x = torch.tensor(up, dtype=torch.float32, device="cuda:0")
    p = molt.make_params(w["eps"], w["dt"], tol=w["tol"], stepper=molt.MOLT_BDF2, max_iter=20000,
                         init=molt.MOLT_INIT_LINEAR, precision=molt.MOLT_F32)
    st, infos = molt.solve(x, g, p, 3)
    e = x.double().cpu().numpy() - ref
    out["patch_vs_oracle"] = {
        "patch": f"{m}x{m} periodic, h = 1/{n}, eps {w['eps']}, BDF2 dt {w['dt']}, tol {w['tol']}, 3 steps",
        "max_abs": float(np.abs(e).max()), "l2": float(np.sqrt((e ** 2).mean())),
        "iters_fp32": [i.iters for i in infos], "iters_oracle": [i.iters for i in rinf]}
    out["target_max_abs"] = 1e-5
    print(f"error: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def run_sweep(molt, n, L, M, launches=20):
    """The standalone line inverse along x and along y of an n x n periodic
    field, FP32 and FP64, timed with events around `launches` back-to-back
    launches on the current stream (one launch = one inverse of every line)."""
    import torch
    out = {}
    g = molt.make_grid(n, n, 0.0, L, 0.0, L, molt.MOLT_BC_PERIODIC, M)
    stream = torch.cuda.current_stream()
    for prec, dt, tag in ((molt.MOLT_F32, torch.float32, "fp32"), (molt.MOLT_F64, torch.float64, "fp64")):
        x = torch.rand(n, n, dtype=dt, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(7))
        y = torch.empty_like(x)
        esz = x.element_size()
        for axis, name in ((0, "x"), (1, "y")):
            need = molt.molt_sweep_workspace_bytes(g, axis, prec, 1)
            work = molt.workspace(need)
            args = (g, axis, 278.3, prec, x.data_ptr(), y.data_ptr(), 1, work.data_ptr(), work.numel(),
                    stream.cuda_stream)
            for _ in range(3):
                molt.mol_t_helmholtz_sweep(*args)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(launches):
                rc = molt.mol_t_helmholtz_sweep(*args)
            ev1.record(stream)
            torch.cuda.synchronize()
            if rc != molt.MOLT_OK:
                raise molt.MoltError(rc, "mol_t_helmholtz_sweep")
            sec = ev0.elapsed_time(ev1) / 1e3 / launches
            byts = n * n * 2 * esz  # read the field once, write it once
            out[f"{name}_{tag}"] = {"gpt_sweeps_per_s": round(n * n / sec / 1e9, 1), "us_per_launch": round(sec * 1e6, 2),
                                    "gb_per_s": round(byts / sec / 1e9, 1),
                                    "frac_of_8tbs": round(byts / sec / 1e9 / HBM_PEAK_GBS, 4)}
            del work
        del x, y
    out["field"] = f"{n}x{n} periodic, alpha = 278.3 (the 4096^2 workload's), M = {M}; bytes = field read + written"
    print(f"sweep: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def run_small(args, molt, synth, oracle):
    """The 1D workload (N = 256, BE, FP64, tol 1e-10, 200 steps) and the 512^2
    Neumann workload (BDF2 dt 5e-5, 2000 steps; FP64, then FP32 with the FP64
    setup phase): steps/s on the GPU and of the oracle on one core and on all
    cores, and their errors."""
    import numpy as np
    import torch
    nthreads = host_threads()
    out = {}
    # ---- 1D
    w = synth.WORKLOADS["ch1d_be_n256"]
    u0 = synth.workload_u0("ch1d_be_n256")
    g = molt.make_grid(w["n"], 1, 0.0, w["L"], 0.0, 1.0, molt.MOLT_BC_PERIODIC, w["M"])
    p = molt.make_params(w["eps"], w["dt"], tol=w["tol"], stepper=molt.MOLT_BE, max_iter=5000,
                         precision=molt.MOLT_F64)
    x = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
    molt.solve(x.clone(), g, p, 2)  # warm-up
    (st, infos), tg = _timed(lambda: molt.solve(x, g, p, w["steps"]))
    og = oracle.Grid(nx=w["n"], bc=oracle.BC_PERIODIC, M=w["M"], x0=0.0, x1=w["L"])
    po = oracle.Params(eps=w["eps"], dt=w["dt"], tol=w["tol"], stepper=oracle.BE, max_iter=5000)
    times = {}
    for th in (1, nthreads):
        oracle.set_threads(th)
        t = time.perf_counter()
        ref, rinf = oracle.solve(og, po, u0, w["steps"])
        times[th] = time.perf_counter() - t
    e = x.cpu().numpy() - ref
    print(f"ch1d: gpu {tg:.2f} s, oracle 1 core {times[1]:.2f} s", file=sys.stderr, flush=True)
    out["ch1d"] = {"workload": "1D CH periodic [0,2pi], N=256, eps 0.05, BE dt 1e-3, tol 1e-10, M=4, 200 steps, FP64",
                   "gpu_steps_per_s": round(w["steps"] / tg, 1), "oracle_steps_per_s_1core": round(w["steps"] / times[1], 1),
                   f"oracle_steps_per_s_{nthreads}cores": round(w["steps"] / times[nthreads], 1),
                   "max_abs_vs_oracle": float(np.abs(e).max()), "l2_vs_oracle": float(np.sqrt((e ** 2).mean())),
                   "same_iterations": [i.iters for i in infos] == [i.iters for i in rinf],
                   "iters_total": int(sum(i.iters for i in infos))}
    # ---- 512^2 Neumann
    w = synth.WORKLOADS["ch2d_neumann_bdf2_512"]
    n = w["n"]
    u0 = synth.workload_u0("ch2d_neumann_bdf2_512")
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_NEUMANN, w["M"])
    nst = args.c2_steps
    fields, rec = {}, {}
    for prec, dt, tol in ((molt.MOLT_F64, torch.float64, 1e-10), (molt.MOLT_F32, torch.float32, 1e-8),
                          ("f64_1e-8", torch.float64, 1e-8)):
        p = molt.make_params(w["eps"], w["dt"], tol=tol, stepper=molt.MOLT_BDF2, max_iter=5000,
                             init=molt.MOLT_INIT_LINEAR, precision=molt.MOLT_F64 if dt == torch.float64 else molt.MOLT_F32)
        x = torch.tensor(u0, dtype=dt, device="cuda:0")
        (st, infos), tg = _timed(lambda: molt.solve(x, g, p, nst))
        fields[prec] = x.double().cpu().numpy()
        it = [i.iters for i in infos]
        print(f"ch2d_neumann: precision {prec}: {nst} steps in {tg:.1f} s, mean iterations {np.mean(it):.1f}",
              file=sys.stderr, flush=True)
        rec[prec] = {"status": st, "gpu_steps_per_s": round(nst / tg, 1), "seconds": round(tg, 2),
                     "iters_first": it[:4], "iters_mean": round(float(np.mean(it)), 1), "iters_max": max(it),
                     "steps_over_300_iters": int(sum(1 for k in it if k > 300)),
                     "energy_first_last": [infos[0].energy, infos[-1].energy],
                     "gpt_sweeps_per_s": round(n * n * sum(4 + 7 * k for k in it) / tg / 1e9, 2)}
    d = fields[molt.MOLT_F32] - fields[molt.MOLT_F64]
    d8 = fields[molt.MOLT_F32] - fields["f64_1e-8"]
    # the oracle: 3 converged steps (all cores, compared with both GPU runs'
    # first 3 steps), and a bounded 1-core sample
    og = oracle.Grid(nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=oracle.BC_NEUMANN, M=w["M"])
    oracle.set_threads(nthreads)
    # (at tol 1e-8: the first steps of the workload need thousands of
    # iterations at 1e-10, too long for the oracle here)
    po = oracle.Params(eps=w["eps"], dt=w["dt"], tol=1e-8, stepper=oracle.BDF2, max_iter=5000,
                       init=oracle.INIT_LINEAR)
    t = time.perf_counter()
    ref, rinf = oracle.solve(og, po, u0, 3)
    t_all = time.perf_counter() - t
    print(f"ch2d_neumann: oracle 3 steps on {nthreads} threads in {t_all:.1f} s", file=sys.stderr, flush=True)
    errs = {}
    for prec, dt in ((molt.MOLT_F64, torch.float64), (molt.MOLT_F32, torch.float32)):
        p = molt.make_params(w["eps"], w["dt"], tol=1e-8, stepper=molt.MOLT_BDF2, max_iter=5000,
                             init=molt.MOLT_INIT_LINEAR, precision=prec)
        x = torch.tensor(u0, dtype=dt, device="cuda:0")
        molt.solve(x, g, p, 3)
        e = x.double().cpu().numpy() - ref
        errs[prec] = {"max_abs": float(np.abs(e).max()), "l2": float(np.sqrt((e ** 2).mean()))}
    oracle.set_threads(1)
    po1 = oracle.Params(eps=w["eps"], dt=w["dt"], stepper=oracle.BE, fixed_iters=10, init=oracle.INIT_LINEAR)
    t = time.perf_counter()
    oracle.step(og, po1, u0)
    t_one = time.perf_counter() - t
    oracle.set_threads(nthreads)
    its = sum(i.iters for i in rinf)
    out["ch2d_neumann"] = {
        "workload": f"2D CH Neumann [0,1]^2, 512x512, eps 0.01, BDF2 dt 5e-5 (BE start-up), M=4, init R, "
                    f"{nst} steps; FP64 tol 1e-10, FP32 tol 1e-8, iteration cap 5000",
        "fp64": rec[molt.MOLT_F64], "fp32": rec[molt.MOLT_F32],
        "fp64_tol_1e-8": rec["f64_1e-8"],
        # the FP32 error proper: against FP64 at the same tolerance; against
        # FP64 at 1e-10 it also holds the tolerance's own error
        "fp32_vs_fp64_same_tol_after_all_steps": {"max_abs": float(np.abs(d8).max()),
                                                  "l2": float(np.sqrt((d8 ** 2).mean()))},
        "fp32_vs_fp64_tol_1e-10_after_all_steps": {"max_abs": float(np.abs(d).max()),
                                                   "l2": float(np.sqrt((d ** 2).mean()))},
        "vs_oracle_after_3_steps_tol_1e-8": {"fp64": errs[molt.MOLT_F64], "fp32": errs[molt.MOLT_F32],
                                             "oracle_iters": [i.iters for i in rinf]},
        "oracle_gpt_sweeps_per_s": {f"{nthreads}cores": round(n * n * (12 + 7 * its) / t_all / 1e9, 4),
                                    "1core": round(n * n * (4 + 7 * 10) / t_one / 1e9, 4)},
        "oracle_steps_per_s": {f"{nthreads}cores (first 3 steps)": round(3 / t_all, 3)},
    }
    print(f"small: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def run_full(args, molt, w, grid, params, u0):
    """The whole workload once: every step from u0 (BE start-up, then BDF2),
    per-step iteration counts and wall time (not the headline value, which
    is timed over the steady steps)."""
    import numpy as np
    import torch
    u = torch.tensor(u0, dtype=torch.float32, device="cuda:0")
    up = torch.empty_like(u)
    work = molt.workspace(molt.ch_workspace_bytes(grid, params))
    stream = torch.cuda.current_stream().cuda_stream
    nsteps = args.full_steps
    its, secs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nsteps):
        params.have_prev = 1 if k > 0 else 0
        info = molt.molt_step_info()
        ts = time.perf_counter()
        rc = molt.ch_step(grid, params, u.data_ptr(), up.data_ptr(), work.data_ptr(), work.numel(), info, stream)
        if rc != molt.MOLT_OK:
            raise molt.MoltError(rc, f"ch_step (full workload, step {k + 1})")
        its.append(info.iters)
        secs.append(time.perf_counter() - ts)
        if (k + 1) % 100 == 0:
            print(f"full workload: {k + 1}/{nsteps} steps, {time.perf_counter() - t0:.2f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pts = float(grid.nx) * grid.ny
    # the same steps in FP64 (the GPU path the tests pin to the oracle at
    # 1e-12 relative): the FP32 result's error after the whole workload
    err = None
    if args.full_fp64:
        p64 = molt.make_params(params.eps, params.dt, tol=params.tol, stepper=params.stepper,
                               max_iter=params.max_iter, init=params.init, precision=molt.MOLT_F64)
        u64 = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
        up64 = torch.empty_like(u64)
        work64 = molt.workspace(molt.ch_workspace_bytes(grid, p64))
        its64 = []
        t64 = time.perf_counter()
        for k in range(nsteps):
            p64.have_prev = 1 if k > 0 else 0
            inf64 = molt.molt_step_info()
            rc = molt.ch_step(grid, p64, u64.data_ptr(), up64.data_ptr(), work64.data_ptr(), work64.numel(), inf64,
                              stream)
            if rc != molt.MOLT_OK:
                raise molt.MoltError(rc, f"ch_step (full workload FP64, step {k + 1})")
            its64.append(inf64.iters)
            if (k + 1) % 100 == 0:
                print(f"full workload FP64: {k + 1}/{nsteps} steps, {time.perf_counter() - t64:.2f} s",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t64
        d = u.double() - u64
        err = {"max_abs": float(d.abs().max()), "l2": float(d.pow(2).mean().sqrt()),
               "fp64_seconds": round(t64, 3), "fp64_iters_mean_after_10": round(float(np.mean(its64[10:] or its64)), 2),
               "steps_with_equal_iteration_counts": int(sum(a == b for a, b in zip(its, its64))),
               "mass_fp32_minus_fp64": info.mass - inf64.mass}
        del u64, up64, work64
    out = {"steps": nsteps, "seconds": round(elapsed, 3), "steps_per_s": round(nsteps / elapsed, 2),
           "gpt_sweeps_per_s": round(pts * sum(4 + 7 * k for k in its) / elapsed / 1e9, 1),
           "iters_first_10": its[:10], "iters_last_10": its[-10:],
           "iters_min_max_mean_after_10": [min(its[10:] or its), max(its[10:] or its),
                                           round(float(np.mean(its[10:] or its)), 2)],
           "ms_per_step_after_10": round(1e3 * float(np.mean(secs[10:] or secs)), 3),
           "mass_last": info.mass, "energy_last": info.energy, "fp32_vs_fp64_after_all_steps": err}
    print(f"full workload: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is design-only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return

    import numpy as np
    import torch

    from paper_1611_04214_amd import molt, synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    molt.load()
    name = "ch2d_periodic_bdf2_4096"
    w = synth.WORKLOADS[name]
    n = args.n
    cls = next(c for c in range(molt.MOLT_TUNE_CLASSES) if n <= (128 << c) or c == molt.MOLT_TUNE_CLASSES - 1)
    if args.shape == "auto":
        molt.autotune(molt.MOLT_F32, n)
    elif args.shape != "default":
        kx, ky = (int(v) for v in args.shape.split(","))
        if molt.molt_tune_set(molt.MOLT_F32, cls, kx, ky) != molt.MOLT_OK:
            raise SystemExit(f"bench.py: shape {args.shape} is not valid for n = {n}")
    shape = molt.molt_tune_get(molt.MOLT_F32, cls)
    grid = molt.make_grid(n, n, 0.0, w["L"], 0.0, w["L"], molt.MOLT_BC_PERIODIC, w["M"])
    init = molt.MOLT_INIT_LINEAR if args.init == "linear" else molt.MOLT_INIT_PREV
    params = molt.make_params(w["eps"], w["dt"], tol=w["tol"], stepper=molt.MOLT_BDF2, max_iter=args.max_iter,
                              init=init, precision=molt.MOLT_F32)
    u0 = synth.workload_u0(name, n)
    u = torch.tensor(u0, dtype=torch.float32, device="cuda:0")
    up = torch.empty_like(u)
    work = molt.workspace(molt.ch_workspace_bytes(grid, params))
    stream = torch.cuda.current_stream().cuda_stream

    def one_step(k: int) -> molt.molt_step_info:
        params.have_prev = 1 if k > 0 else 0
        info = molt.molt_step_info()
        rc = molt.ch_step(grid, params, u.data_ptr(), up.data_ptr(), work.data_ptr(), work.numel(), info, stream)
        if rc < 0:
            raise molt.MoltError(rc, "ch_step")
        return info

    step_idx = 0
    warm = []
    warm_prof = {}
    for k in range(args.warmup):
        # the last warm-up step times every kernel (per-kernel breakdown, and the
        # dominant kernel); the timed steps then time that kernel alone, since
        # the events around every launch would slow the stream measurably
        last = k == args.warmup - 1 and not args.no_profile
        if last:
            molt.molt_profile_only(-1)
            molt.molt_profile(1)
        t = time.perf_counter()
        inf = one_step(step_idx)
        step_idx += 1
        warm.append((inf.iters, time.perf_counter() - t))
        if last:
            warm_prof = molt.molt_profile_read()
            molt.molt_profile(0)
        print(f"warmup step {step_idx}: iters={inf.iters} residual={inf.residual:.3e} "
              f"time={warm[-1][1]:.3f}s", file=sys.stderr, flush=True)

    if not args.no_profile:
        dom_w = max((k for k in warm_prof if k in BYTES_PER_POINT), key=lambda k: warm_prof[k][1], default=None)
        molt.molt_profile_only(molt.kind_of(dom_w) if dom_w is not None else -1)
        molt.molt_profile(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(one_step(step_idx))
        step_idx += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k, inf in enumerate(infos):  # (printed after the timed region)
        print(f"timed step {step_idx - len(infos) + k + 1}: iters={inf.iters} residual={inf.residual:.3e}",
              file=sys.stderr, flush=True)
    prof = molt.molt_profile_read() if not args.no_profile else {}
    molt.molt_profile(0)
    molt.molt_profile_only(-1)

    elapsed = t1 - t0
    iters = [i.iters for i in infos]
    pts = float(n) * n
    executed = pts * sum(4 + 7 * k for k in iters)
    nominal = pts * sum(4 + 8 * k for k in iters)
    value = executed / elapsed / 1e9

    roof = None
    # per-kernel breakdown: the last warm-up step (every kernel timed), else
    # the timed steps when there was no warm-up
    every = warm_prof or prof
    # launches queued after convergence exit at once: the FP32 iteration
    # kinds are averaged over the iterations that ran (their total time
    # includes the no-op launches: pessimistic), the others over launches
    real_w = max(warm[-1][0] - 1 - (warm[-1][0] - 1) // 64, 1) if warm else max(sum(iters) - len(iters), 1)
    kernels = {kname: {"launches": launches,
                       "avg_us": 1e3 * ms / (real_w if kname in BYTES_PER_POINT else max(launches, 1))}
               for kname, (launches, ms) in every.items()}
    if prof:
        nsteps = len(infos)
        table = BYTES_PER_POINT
        dom = max((k for k in prof if k in table), key=lambda k: prof[k][1], default=None)
        if dom is not None:
            # the FP32 kernels run the increment-form iterations (each step's
            # first iteration runs in FP64, timed under the f64_ kinds); one
            # launch of each pass per iteration did work, launches queued after
            # convergence exit at once and their (small) time is left in the
            # total (pessimistic)
            _, ms = prof[dom]
            # FP32 iterations: all but each step's first and its FP64 restarts
            # (every 64th)
            real = sum(k - 1 - (k - 1) // 64 for k in iters)
            per_launch = pts * table[dom]
            avg_s = ms / 1e3 / real
            achieved = per_launch / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(dom, n),
                    "kernel": dom,
                    "bytes_per_launch": per_launch, "avg_launch_us": round(avg_s * 1e6, 2)}
            total_ms = sum(v[1] for v in every.values())
            roof["kernel_share_of_gpu_time"] = (round(every[dom][1] / total_ms, 3)
                                                if total_ms > 0 and dom in every else None)
            roof["timed_in_timed_steps"] = sorted(prof)
    if warm_prof:
        # the whole FP32 iteration: every field read once and written once
        # (ITER_BYTES_PER_POINT) over the summed time of the iteration's FP32
        # kernels in the last warm-up step (which timed every kernel)
        it_kinds = [k for k in warm_prof if k in BYTES_PER_POINT or k == "other_sweep"]
        it_ms = sum(warm_prof[k][1] for k in it_kinds)
        if it_ms > 0 and real_w > 0:
            per_it_s = it_ms / 1e3 / real_w
            gbs = float(n) * n * ITER_BYTES_PER_POINT / per_it_s / 1e9
            whole = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_point": ITER_BYTES_PER_POINT,
                     "kernel_us_per_iteration": round(per_it_s * 1e6, 2),
                     "kernels": sorted(it_kinds),
                     "moved_bytes_per_point": sum(BYTES_PER_POINT[k] for k in BYTES_PER_POINT if k in warm_prof)}
            wall_us = 1e6 * elapsed / max(sum(iters), 1)
            whole["wall_us_per_iteration_timed_steps"] = round(wall_us, 2)
            if roof is None:
                roof = {}
            roof["whole_iteration"] = whole

    full = run_full(args, molt, w, grid, params, u0) if args.full_steps > 0 else None

    import oracle
    oracle.build(force=False)
    error = run_error(molt, synth, oracle, w, n) if not args.no_error else None
    sweep = run_sweep(molt, n, w["L"], w["M"]) if not args.no_sweep else None
    small = run_small(args, molt, synth, oracle) if not args.no_small else None
    batched = run_batched(args, molt, synth) if args.batch_steps > 0 else None
    served = run_served(args, molt, synth) if args.serve_count > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        og = oracle.Grid(nx=n, ny=n, x0=0.0, x1=w["L"], y0=0.0, y1=w["L"], bc=oracle.BC_PERIODIC, M=w["M"])
        model, ncpu = cpu_info()
        legs = {}
        for th, its in ((host_threads(), args.cpu_iters), (1, max(2, args.cpu_iters // 8))):
            used = oracle.set_threads(th)
            po = oracle.Params(eps=w["eps"], dt=w["dt"], stepper=oracle.BE, fixed_iters=its,
                               init=oracle.INIT_LINEAR if init == molt.MOLT_INIT_LINEAR else oracle.INIT_PREV)
            tc = time.perf_counter()
            oracle.step(og, po, u0, None)
            tcpu = time.perf_counter() - tc
            legs[used] = (pts * (4 + 7 * its) / tcpu / 1e9, its, tcpu)
        oracle.set_threads(host_threads())
        allc = max(legs)
        v, its, tcpu = legs[allc]
        v1, its1, t1c = legs[1]
        cpu = {"value": round(v, 4), "unit": "Gpt-sweeps/s", "cores": allc, "kind": "oracle",
               "sample": f"first BE step of the {n}^2 workload with {its} fixed-point iterations "
                         f"(4 + 7 per iteration point-sweeps per point), FP64 oracle, {tcpu:.1f} s on {allc} threads",
               "single_core": {"value": round(v1, 4), "iterations": its1, "seconds": round(t1c, 1)},
               "cpu_model": model, "logical_cpus": ncpu}

    out = {
        "metric": "2D CH Gpt-sweeps/s (% HBM peak) + steps/s vs plain path; served p50/p99",
        "value": round(value, 3),
        "unit": "Gpt-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D CH periodic {n}x{n} on [0,1]^2, eps=0.005, BDF2 dt=1e-5, tol 1e-8, M=4, "
                               f"FP32 sweeps, u0=0.3+0.05N(0,1), init={args.init}",
                   "grid": [n, n], "steps_in_workload": w["steps"], "parallelism": "single GPU",
                   "line_block_shape": {"kx": shape[0], "ky": shape[1], "chosen": args.shape}},
        "steps_per_s": round(args.steps / elapsed, 4),
        "iters_per_step": iters,
        "warmup_iters": [k for k, _ in warm],
        "point_iters_per_s": round(pts * sum(iters) / elapsed / 1e9, 3),
        "gpt_sweeps_nominal_8_per_iter": round(nominal / elapsed / 1e9, 3),
        "roofline": roof,
        "cpu_baseline": cpu,
        "error": error,
        "full_workload": full,
        "sweep": sweep,
        "ch1d": small["ch1d"] if small else None,
        "ch2d_neumann": small["ch2d_neumann"] if small else None,
        "batched": batched,
        "served": served,
        "kernels": kernels,
    }
    # leave nothing behind: device memory released and the stream drained
    # before the line is printed
    del u, up, work
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
