"""Benchmark of the augmented Lagrangian OF-DFT hot path on one MI355X.

Default (--mode hotpath, --workload fcc10): the 4000-atom Al-like cluster (10^3 fcc cells,
a = 7.6 Bohr, seeded 0.1 Bohr displacements, 8 Bohr vacuum, h = 0.5 Bohr: 185^3 nodes),
order-12 stencil, Gaussian pseudocharges (Z = 3, s = 1), TFW + LDA, multipole boundary
values, in the precision that configuration names: FP32 stencil and CG vectors inside an
FP64 iterative-refinement Poisson solve.  One step is one pass of the whole hot path from
the atomic-density guess already resident in HBM: the pseudocharge and self energy of the
4000 nuclei, the density and its multipole moments, the boundary fold, the Poisson solve
from zero to 1e-10, the residual and energy pass, two nonlinear-CG steps (each a line
search whose trial points re-solve Poisson warm-started), the multiplier update and the
Hellmann-Feynman forces (alofdft_solve_device with max_outer = 1, max_inner = 2).  The same
pass in FP64 is timed afterwards for the speedup and the error of the refined path.

The JSON line: value = stencil point updates per second over the timed steps (every stencil
application of the pass, FP32 and FP64, times the nodes, over the wall time);
stencil_streaming_185 = the plain stencil alone over six rotating buffer pairs (more than
the 256 MB Infinity Cache) with 16 / 8 bytes per point; roofline = the dominant kernel pair,
one FP32 CG iteration (the stencil launch and the x, r update launch), at 40 bytes per node
(the algorithmic traffic of a fused CG iteration in FP32), over the mean kernel time of the
sampled iterations (HIP events stamped by the runtime on both launches); cpu_baseline = the
oracle's CG iterations on the same grid and right-hand side, all host threads and one.

Other modes: ground_state (time to converged energy and forces, FP32-refined and FP64),
stencil (plain stencil only, then a reference copy for counter calibration), counters (a
short refined Poisson solve, then the reference copy), serve (the 64-request stream of fcc
1-3 clusters at arrival rates 0.5, 1 and 2 times the sequential FP64 capacity), relax,
methods (augmented Lagrangian, penalty and Lagrange multiplier, and the eta0 / mu0 / kappa
sweep), large (the 97 556-atom cluster: pseudocharge, Poisson solves, one hot-path pass per
precision, stencil), --summarize-counters (writes
profiles/traffic.json from two counter CSVs of --mode counters).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "Gpts/s stencil (%HBM peak); AL-OFDFT solves/s, p50/p99 latency vs FP64"
# algorithmic bytes per node: a stencil application reads x once and writes y once; a CG
# iteration is counted as ten array passes, 8 reads and 2 writes of a fused iteration (the
# two launches make 11 in FP32: read r, p, A p and write p, A p, then read x, r, p, A p and
# write x, r; 10 in FP64, whose first launch also makes the previous x += alpha p)
STENCIL_BYTES = {8: 16, 4: 8}
CG_ITER_BYTES = {8: 80, 4: 40}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fcc10", choices=["single", "fcc2", "fcc5", "fcc10"])
    ap.add_argument("--precision", default="auto", choices=["auto", "fp32r", "fp64"],
                    help="auto: the workload's specified precision (FP32-refined for fcc5 and fcc10, "
                         "FP64 for the single atom and fcc2)")
    ap.add_argument("--inner", type=int, default=2, help="hotpath: nonlinear-CG steps per pass")
    ap.add_argument("--no-other-precision", action="store_true", help="skip the pass in the other precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="length of each oracle sample")
    ap.add_argument("--sample-every", type=int, default=16,
                    help="CG iterations per timed sample (an event-stamped launch costs a few us more)")
    ap.add_argument("--cg-schedule", type=int, default=-1, choices=[-1, 0, 1, 2])
    ap.add_argument("--mode", default="hotpath",
                    choices=["hotpath", "ground_state", "stencil", "counters", "serve", "relax", "methods", "large"])
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KEY"),
                    help="write profiles/traffic.json entry KEY from two rocprofv3 counter CSVs of --mode counters")
    ap.add_argument("--requests", type=int, default=64, help="serve: number of requests")
    ap.add_argument("--rate-factors", default="0.5,1,2",
                    help="serve: arrival rates as multiples of the sequential FP64 service rate")
    ap.add_argument("--slots", type=int, default=4, help="serve: concurrent request slots")
    ap.add_argument("--slot-blocks", default="256",
                    help="serve: workgroups per stencil launch of each slot (the server default 256; 0: one round), comma list")
    return ap.parse_args()


def specified_precision(lib, S, precision):
    if precision == "fp32r":
        return lib.FP32_REFINED
    if precision == "fp64":
        return lib.FP64
    return lib.FP32_REFINED if S.name in ("fcc5", "fcc10") else lib.FP64


# ----------------------------------------------------------------- counter summaries
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_digest():
    """Hash of the kernel sources (a counter summary is valid only for the source it was taken on)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("kernels.h", "stencil_inst.hip", "launch.h", "common.h"):
        with open(os.path.join(ROOT, "paper_1405_6456_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(key, path=TRAFFIC_JSON):
    """Fabric bytes per CG iteration from the committed counter summary, if it was taken on
    the current kernel source; else None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ent = json.load(f).get(key)
    if not ent or ent.get("kernels_sha256_16") != kernel_digest():
        return None
    return ent.get("bytes_per_iteration")


def summarize_counters(fetch_csv, write_csv, key, path=TRAFFIC_JSON):
    """Bytes per CG iteration of the FP32 CG kernels (the stencil launch k_stencil2<float, ...,
    CGP1LIOp> -- CGP1LOp<float> before p and A p were interleaved -- and the update
    k_cg_update<float>) from a FETCH_SIZE pass and a WRITE_SIZE
    pass (KiB per dispatch) of --mode counters, each scaled by what the same counter reads for
    the reference copy of 256 MiB in that run (FETCH_SIZE counts a 128-byte read request of
    this part as 64 bytes: its copy reads 128 MiB of the 256).  Updates profiles/traffic.json."""
    import csv

    def per_kernel(csv_path, counter):
        out = {}
        with open(csv_path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    copy_bytes = 256 * 1024 * 1024
    res = {}
    for csv_path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        pk = per_kernel(csv_path, counter)
        st = [v for k, vs in pk.items() if ("CGP1LOp<float>" in k or "CGP1LIOp" in k) and "k_stencil" in k
              for v in vs]
        up = [v for k, vs in pk.items() if "k_cg_update<float" in k for v in vs]
        cp = [v for k, vs in pk.items() if "copyBuffer" in k or "elementwise" in k for v in vs]
        cp = [v for v in cp if v > 0.5 * max(cp)] if cp else []
        if not st or not up or not cp:
            raise SystemExit(f"{csv_path}: no CG or copy dispatches with {counter}")
        scale = copy_bytes / (sum(cp) / len(cp) * 1024.0)
        kst, kup = sum(st) / len(st), sum(up) / len(up)
        res[counter] = {"stencil_kib_per_dispatch": round(kst, 1), "update_kib_per_dispatch": round(kup, 1),
                        "copy_kib": round(sum(cp) / len(cp), 1), "scale": round(scale, 4),
                        "bytes_per_iteration": round((kst + kup) * 1024.0 * scale)}
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[key] = {"kernels_sha256_16": kernel_digest(),
                 "bytes_per_iteration": res["FETCH_SIZE"]["bytes_per_iteration"] +
                 res["WRITE_SIZE"]["bytes_per_iteration"],
                 "read_bytes": res["FETCH_SIZE"]["bytes_per_iteration"],
                 "write_bytes": res["WRITE_SIZE"]["bytes_per_iteration"], "counters": res}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps(data[key]))


# ----------------------------------------------------------------- CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, seconds):
    """The oracle's conjugate-gradient Poisson iterations on the workload's grid and right-hand
    side (u0^2 + b with the multipole boundary values), as stencil point updates per second,
    with all host threads and with one; each sample takes about `seconds`."""
    import oracle
    from paper_1405_6456_amd import synth

    u0 = synth.atomic_guess(system)
    b = oracle.pseudocharge(system)
    rhs = oracle.poisson_rhs(system.grid, 6, 1, u0 * u0 + b)
    pts = system.grid.npts

    def rate():
        t = time.perf_counter()
        oracle.poisson_cg(system.grid, 6, rhs, tol=1e-300, maxit=2)
        per = (time.perf_counter() - t) / 3.0  # initial residual + 2 iterations
        iters = max(2, int(seconds / max(per, 1e-6)))
        t = time.perf_counter()
        _, it, _, _ = oracle.poisson_cg(system.grid, 6, rhs, tol=1e-300, maxit=iters)
        dt = time.perf_counter() - t
        return (it + 1) * pts / dt / 1e9, it, dt

    threads = oracle.get_threads()
    v_all, it_all, dt_all = rate()
    oracle.set_threads(1)
    v_one, it_one, dt_one = rate()
    oracle.set_threads(threads)
    return {"value": v_all, "unit": "Gpts/s", "cores": threads, "kind": "oracle", "value_1thread": v_one,
            "cpu_model": cpu_model(),
            "sample": f"oracle CG Poisson on the {system.name} grid ({pts} nodes): {it_all} iterations + initial "
                      f"residual in {dt_all:.1f} s on {threads} threads, {it_one} in {dt_one:.1f} s on one "
                      f"(stencil point updates per second of the same operator)"}


# ----------------------------------------------------------------- helpers
def stencil_streaming(ctx, n, reps=50):
    """Plain stencil over six rotating buffer pairs, FP64 and FP32: Gpts/s and the fraction of
    the HBM peak at 16 / 8 bytes per point."""
    npts = n[0] * n[1] * n[2]
    out = {}
    for dt, name, es in ((0, "f64", 8), (1, "f32", 4)):
        ms = ctx.bench_stencil(n, 6, dt, reps=reps, nbuf=6)
        out[name] = {"ms": round(ms, 5), "gpts": round(npts / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(npts * STENCIL_BYTES[es] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def cg_roofline(ctx, lib, prec, key):
    """The dominant kernel pair of the pass: one CG iteration of the precision's inner solve."""
    dt_idx = 1 if prec == lib.FP32_REFINED else 0
    es = 4 if prec == lib.FP32_REFINED else 8
    n, ms, pts, sched, first, second = ctx.cg_kernel_stats(dt_idx, split=True)
    alg = CG_ITER_BYTES[es] * pts
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    names = {0: "k_stencil2<CGP1Op> + k_cg_update",
             1: "k_stencil2<CGP1LIOp> + k_cg_update" if es == 4 else "k_stencil2<CGP1LOp> + k_cg_update",
             2: "k_stencil2<CGPipeOp>"}
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(key),
            "kernel": f"CG iteration ({'FP32' if es == 4 else 'FP64'}): {names.get(sched, '?')}",
            "alg_bytes_per_iteration": alg, "mean_iteration_ms": round(ms, 5),
            "first_launch_ms": round(first, 5), "second_launch_ms": round(second, 5), "timed_iterations": n,
            "schedule": sched}


# ----------------------------------------------------------------- modes
def hotpath(args):
    import numpy as np
    import torch

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    S = synth.config(args.workload)
    npts = S.grid.npts
    prec = specified_precision(lib, S, args.precision)
    ctx = lib.Context(0)
    ctx.set_cg_schedule(args.cg_schedule)
    guess = lib.default_params(initial_guess=lib.GUESS_ATOMIC)
    u0 = ctx.initial_guess(S, guess)  # resident in HBM before the timed region
    step_prm = lambda p: lib.default_params(precision=p, max_outer=1, max_inner=args.inner)

    for _ in range(args.warmup):
        ctx.solve_device(S, step_prm(prec), u0, want_forces=True)
    ctx.profile_cg_kernel(args.sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [ctx.solve_device(S, step_prm(prec), u0, want_forces=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    key = f"cg_{'f32' if prec == lib.FP32_REFINED else 'f64'}_{S.name}"
    roofline = cg_roofline(ctx, lib, prec, key)
    ctx.profile_cg_kernel(0)
    last = outs[-1]
    mv = sum(o["matvec_fp64"] + o["matvec_fp32"] for o in outs)
    line = {
        "metric": METRIC,
        "value": round(mv * npts / wall / 1e9, 2),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 stencil/CG + f64 refinement" if prec == lib.FP32_REFINED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{S.name}: {S.M}-atom Al-like fcc cluster, {S.grid.n[0]}^3 nodes, h={S.grid.h}, "
                               f"order 12, {'FP32 CG + FP64 refinement' if prec == lib.FP32_REFINED else 'FP64'}"
                               f"; one hot-path pass per step (setup, {args.inner} nonlinear-CG steps, forces)",
                   "atoms": S.M, "nodes": npts, "parallelism": "single GPU"},
        "counts": {k: last[k] for k in ("outer", "inner", "grad_evals", "poisson_solves", "cg_iters", "matvec_fp64",
                                        "matvec_fp32", "refinements")},
        "E_total": last["E_total"],
    }
    if not args.no_other_precision:
        other = lib.FP64 if prec == lib.FP32_REFINED else lib.FP32_REFINED
        ctx.solve_device(S, step_prm(other), u0, want_forces=True)
        ctx.profile_cg_kernel(args.sample_every)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 3
        oth = [ctx.solve_device(S, step_prm(other), u0, want_forces=True) for _ in range(reps)][-1]
        torch.cuda.synchronize()
        t_oth = (time.perf_counter() - t) / reps
        okey = f"cg_{'f32' if other == lib.FP32_REFINED else 'f64'}_{S.name}"
        oroof = cg_roofline(ctx, lib, other, okey)
        ctx.profile_cg_kernel(0)
        t_main = wall / args.steps
        r32, r64 = (last, oth) if prec == lib.FP32_REFINED else (oth, last)
        t32, t64 = (t_main, t_oth) if prec == lib.FP32_REFINED else (t_oth, t_main)
        line["other_precision_pass"] = {"dtype": "f64" if other == lib.FP64 else "f32r", "ms_per_step":
                                        round(1e3 * t_oth, 2), "cg_iters": oth["cg_iters"], "roofline": oroof}
        line["speedup_fp32r_vs_fp64"] = round(t64 / t32, 3)
        line["err_fp32r_vs_fp64"] = {"E_per_atom": abs(r32["E_total"] - r64["E_total"]) / S.M,
                                     "F_max": float(np.abs(r32["forces"] - r64["forces"]).max())}
    line["stencil_streaming_185"] = stencil_streaming(ctx, synth.config("fcc10").grid.n)
    line["roofline"] = roofline
    line["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(S, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


def ground_state(args):
    """Time to converged energy and forces on the workload, FP32-refined and FP64, from the
    atomic-density guess; the error of the refined result against the FP64 one."""
    import numpy as np
    import torch

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    S = synth.config(args.workload)
    ctx = lib.Context(0)
    u0 = ctx.initial_guess(S, lib.default_params(initial_guess=lib.GUESS_ATOMIC))
    res = {}
    for name, prec in (("f32r", lib.FP32_REFINED), ("f64", lib.FP64)):
        ctx.profile_cg_kernel(args.sample_every)
        torch.cuda.synchronize()
        t = time.perf_counter()
        o = ctx.solve_device(S, lib.default_params(precision=prec), u0, want_forces=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        roof = cg_roofline(ctx, lib, prec, f"cg_{'f32' if prec == lib.FP32_REFINED else 'f64'}_{S.name}")
        ctx.profile_cg_kernel(0)
        res[name] = o
        print(json.dumps({"mode": "ground_state", "workload": S.name, "precision": name, "status": o["status"],
                          "wall_s": round(wall, 2), "E_total": o["E_total"], "E_per_atom": o["E_total"] / S.M,
                          "outer": o["outer"], "inner": o["inner"], "cg_iters": o["cg_iters"],
                          "matvecs": o["matvec_fp64"] + o["matvec_fp32"], "grad_norm": o["grad_norm"],
                          "gpts": round((o["matvec_fp64"] + o["matvec_fp32"]) * S.grid.npts / wall / 1e9, 1),
                          "roofline": roof}), flush=True)
    print(json.dumps({"mode": "ground_state", "workload": S.name,
                      "err_fp32r_vs_fp64": {"E_per_atom": abs(res["f32r"]["E_total"] - res["f64"]["E_total"]) / S.M,
                                            "F_max": float(np.abs(res["f32r"]["forces"] - res["f64"]["forces"]).max())}}),
          flush=True)
    ctx.close()


def fifo_latencies(arrivals, service):
    """Single-server FIFO queue: latency (finish - arrival) of each request."""
    t, out = 0.0, []
    for a, s in zip(arrivals, service):
        t = max(t, a) + s
        out.append(t - a)
    return out


def pct(v, q):
    import math

    v = sorted(v)
    k = max(1, math.ceil(q * len(v)))
    return v[min(len(v), k) - 1]


def serve(args):
    """Request stream: fcc m^3 clusters, m ~ U{1,2,3} (seed 2014), displacement seed 10000+k,
    Poisson arrivals (seed 2015) at f x the sequential FP64 service rate for each f of
    --rate-factors; served with FP32-refined solves (the stream's specified precision) through
    the serving loop, against a FIFO replay of the same arrivals with the measured sequential
    FP64 service times.  One JSON line per f."""
    import threading

    import numpy as np

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    reqs = synth.serving_requests(args.requests)
    ms = [round((S.M // 4) ** (1 / 3)) for S in reqs]
    ctx = lib.Context(0)
    prm64 = lib.default_params(initial_guess=lib.GUESS_ATOMIC)
    prm32 = lib.default_params(precision=lib.FP32_REFINED, initial_guess=lib.GUESS_ATOMIC)
    ctx.solve(reqs[0], prm64, None, want_fields=False)  # warm-up
    first = {}
    for k, m in enumerate(ms):
        first.setdefault(m, k)
    svc64, ref = {}, {}
    for m, k in sorted(first.items()):
        t = time.perf_counter()
        ref[m] = ctx.solve(reqs[k], prm64, None, want_fields=False)
        svc64[m] = time.perf_counter() - t
    service = [svc64[m] for m in ms]
    c_seq = 1.0 / (sum(service) / len(service))
    for f, sb in [(float(x), int(y)) for x in args.rate_factors.split(",") for y in args.slot_blocks.split(",")]:
        rate = f * c_seq
        arrivals = synth.arrival_times(len(reqs), rate)
        seq_lat = fifo_latencies(list(arrivals), service)
        srv = lib.Server(0, max_slots=args.slots)
        srv.set_tuning(sb)
        tickets = [None] * len(reqs)
        t0 = time.perf_counter()

        def submitter():
            for k, S in enumerate(reqs):
                d = arrivals[k] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                tickets[k] = srv.submit(S, prm32)

        th = threading.Thread(target=submitter)
        th.start()
        results = [None] * len(reqs)
        pending = set(range(len(reqs)))
        while pending:
            for k in list(pending):
                if tickets[k] is not None:
                    r = srv.poll(tickets[k])
                    if r is not None:
                        results[k] = r
                        pending.discard(k)
                        done = len(reqs) - len(pending)
                        if done % 16 == 0:
                            print(f"serve f={f}: {done}/{len(reqs)} completed at {time.perf_counter() - t0:.1f} s",
                                  file=sys.stderr, flush=True)
            time.sleep(0.005)
        th.join()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        print(f"serve f={f} slot blocks {sb}: {st['completed']} done in {wall:.1f} s", file=sys.stderr, flush=True)
        err_e = max(abs(results[k]["E_total"] - ref[m]["E_total"]) / reqs[k].M for m, k in first.items())
        err_f = max(float(np.abs(results[k]["forces"] - ref[m]["forces"]).max()) for m, k in first.items())
        print(json.dumps({
            "metric": METRIC, "mode": "serve", "value": round(st["solves_per_s"], 4), "unit": "solves/s",
            "n_gpus": 1, "higher_is_better": True, "dtype": "f32 stencil/CG + f64 refinement", "data": "synthetic",
            "config": {"workload": f"serving stream: {len(reqs)} fcc m^3 clusters, m in {{1,2,3}} (48^3..79^3 nodes),"
                                   f" Poisson arrivals at {f} x the sequential FP64 rate", "slots": args.slots,
                       "slot_blocks": sb},
            "served": {"p50_ms": round(st["p50_ms"], 1), "p99_ms": round(st["p99_ms"], 1),
                       "mean_ms": round(st["mean_ms"], 1), "solves_per_s": round(st["solves_per_s"], 4),
                       "wall_s": round(wall, 1), "completed": st["completed"],
                       "statuses": sorted(set(r["status"] for r in results))},
            "sequential_fp64": {"p50_ms": round(1e3 * pct(seq_lat, 0.5), 1), "p99_ms": round(1e3 * pct(seq_lat, 0.99), 1),
                                "service_s": {str(m): round(v, 3) for m, v in svc64.items()},
                                "capacity_solves_per_s": round(c_seq, 4)},
            "arrival_rate_per_s": round(rate, 4),
            "err_vs_fp64": {"E_per_atom": err_e, "F_max": err_f}}), flush=True)
    ctx.close()


def methods_mode():
    """The paper's method comparison on the synthetic workloads (Sec. 5.3): the augmented
    Lagrangian, the penalty method (eta fixed at 0) and the Lagrange-multiplier method on the
    single atom and the 32-atom cluster, and the augmented Lagrangian's sensitivity to eta0,
    mu0 and kappa on the 32-atom cluster -- stencil applications (the paper's cost measure),
    iterations, energy, time.  FP64."""
    import torch

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    ctx = lib.Context(0)

    def run(name, quiet=False, **kw):
        S = synth.config(name)
        prm = lib.default_params(precision=lib.FP64, **kw)
        u0 = ctx.initial_guess(S, lib.default_params(initial_guess=lib.GUESS_ATOMIC if name != "single" else
                                                     lib.GUESS_UNIFORM))
        torch.cuda.synchronize()
        t = time.perf_counter()
        o = ctx.solve_device(S, prm, u0, want_forces=False)
        wall = time.perf_counter() - t
        if not quiet:
            print(json.dumps({"mode": "methods", "workload": name, **kw, "status": o["status"],
                              "matvecs": o["matvec_fp64"], "outer": o["outer"], "inner": o["inner"],
                              "E_per_atom": o["E_total"] / S.M, "eta_star": o["eta_star"],
                              "grad_norm": o["grad_norm"], "C_h_per_N": o["C_h"] / S.N,
                              "wall_s": round(wall, 3)}), flush=True)
        return o

    run("single", quiet=True)  # warm-up
    for name in ("single", "fcc2"):
        for method in (lib.AL, lib.PENALTY, lib.LAGRANGE):
            run(name, method=method)
    for eta0, mu0, kappa in ((0.0, 1.0, 0.1), (-0.4, 1.0, 0.1), (-0.2, 0.1, 0.1), (-0.2, 10.0, 0.1),
                             (-0.2, 1.0, 0.01), (-0.2, 1.0, 0.5)):
        run("fcc2", eta0=eta0, mu0=mu0, kappa=kappa)
    ctx.close()


def large_mode():
    """The size of the paper's largest cluster on one device: 29^3 fcc cells (97 556 atoms),
    474^3 = 106.5 M nodes: the pseudocharge of all atoms, Poisson solves (multipole boundary
    values, 1e-10, from zero) of u0^2 + b with the atomic-density guess in FP64 and
    FP32-refined with their CG-iteration roofline, one pass of the hot path (as the default
    line: one AL step with two nonlinear-CG steps, energies and forces) in both precisions
    with their agreement, and the plain stencil at that size."""
    import torch

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    S = synth.config("fcc29")
    g = S.grid
    ctx = lib.Context(0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    b, _ = ctx.pseudocharge(S)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "large", "step": "pseudocharge", "atoms": S.M, "nodes": g.npts,
                      "ms": round(1e3 * (time.perf_counter() - t), 1),
                      "neutrality": float(g.h ** 3 * b.sum().item() + S.Z.sum())}), flush=True)
    u0 = ctx.initial_guess(S, lib.default_params(initial_guess=lib.GUESS_ATOMIC))
    rho = (u0 * u0 + b).contiguous()
    del u0
    for prec, name in ((lib.FP64, "f64"), (lib.FP32_REFINED, "f32r")):
        ctx.profile_cg_kernel(64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        phi, its, rel = ctx.poisson(rho, g, bc=lib.BC_MULTIPOLE, precision=prec, tol=1e-10)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        roof = cg_roofline(ctx, lib, prec, f"cg_{'f32' if prec == lib.FP32_REFINED else 'f64'}_fcc29")
        ctx.profile_cg_kernel(0)
        print(json.dumps({"mode": "large", "step": f"poisson_{name}", "cg_iters": its, "relres": rel,
                          "wall_s": round(wall, 3), "us_per_iter": round(1e6 * wall / max(1, its), 1),
                          "roofline": roof}), flush=True)
        del phi
    del rho, b
    u0 = ctx.initial_guess(S, lib.default_params(initial_guess=lib.GUESS_ATOMIC))
    res = {}
    for prec, name in ((lib.FP32_REFINED, "f32r"), (lib.FP64, "f64")):
        ctx.profile_cg_kernel(64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        o = ctx.solve_device(S, lib.default_params(precision=prec, max_outer=1, max_inner=2), u0, want_forces=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        roof = cg_roofline(ctx, lib, prec, f"cg_{'f32' if prec == lib.FP32_REFINED else 'f64'}_fcc29")
        ctx.profile_cg_kernel(0)
        res[name] = o
        mv = o["matvec_fp64"] + o["matvec_fp32"]
        print(json.dumps({"mode": "large", "step": f"pass_{name}", "wall_s": round(wall, 3),
                          "gpts": round(mv * g.npts / wall / 1e9, 2), "E_per_atom": o["E_total"] / S.M,
                          "inner": o["inner"], "poisson_solves": o["poisson_solves"], "cg_iters": o["cg_iters"],
                          "roofline": roof}), flush=True)
    print(json.dumps({"mode": "large", "step": "pass_agreement",
                      "E_per_atom": abs(res["f32r"]["E_total"] - res["f64"]["E_total"]) / S.M,
                      "F_max": float(abs(res["f32r"]["forces"] - res["f64"]["forces"]).max())}), flush=True)
    del u0
    print(json.dumps({"mode": "large", "step": "stencil", **stencil_streaming(ctx, g.n, reps=10)}), flush=True)
    ctx.close()


def relax_mode():
    """Relaxation of the two-atom analogue of the paper's Al2 case (Z = 3, Gaussian
    pseudocharges, 27^3 nodes at h = 0.9 Bohr) from 4.0 Bohr apart to ftol = 2e-4 Ha/Bohr."""
    import numpy as np
    import torch

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    n, h = 27, 0.9
    g = synth.Grid((n, n, n), h, (0.0, 0.0, 0.0))
    c = 0.5 * (n - 1) * h
    R = np.array([[c, c, c - 2.0], [c + 0.05, c - 0.1, c + 2.0]])
    S = synth.System("pair", g, R, np.array([3.0, 3.0]), 6.0)
    ctx = lib.Context(0)
    u0 = synth.initial_u(g, S.N)
    ctx.solve(S, lib.default_params(), u0, want_fields=False)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = ctx.relax(S, lib.default_params(), lib.default_relax_params(ftol=2e-4), u0)
    wall = time.perf_counter() - t
    d = float(np.linalg.norm(out["R"][1] - out["R"][0]))
    print(json.dumps({"mode": "relax", "workload": "pair, Z=3, 27^3 nodes, h=0.9, from 4.0 Bohr, ftol 2e-4",
                      "wall_s": round(wall, 3), "steps": out["steps"], "solves": out["solves"],
                      "ms_per_solve": round(1e3 * wall / max(1, out["solves"]), 1), "fmax": out["fmax"],
                      "bond_bohr": round(d, 4), "E_total": out["E_total"], "status": out["relax_status"]}),
          flush=True)
    ctx.close()


def reference_copy():
    """A 256 MiB device-to-device copy, whose counter readings calibrate the byte counters."""
    import torch

    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"reference_copy_bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8}), flush=True)


def counters_mode(args):
    """A short Poisson solve on the workload grid in its specified precision (its CG kernels
    are the ones of interest), then the reference copy."""
    import torch

    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    S = synth.config(args.workload)
    ctx = lib.Context(0)
    ctx.set_cg_schedule(args.cg_schedule)
    u0 = ctx.initial_guess(S, lib.default_params(initial_guess=lib.GUESS_ATOMIC))
    b, _ = ctx.pseudocharge(S)
    rho = (u0 * u0 + b).contiguous()
    _, its, rel = ctx.poisson(rho, S.grid, precision=specified_precision(lib, S, args.precision), tol=1e-10,
                              max_cg=200)
    torch.cuda.synchronize()
    print(json.dumps({"workload": S.name, "cg_iters": its, "relres": rel}), flush=True)
    ctx.close()
    reference_copy()


def stencil_mode(args):
    import paper_1405_6456_amd as lib
    from paper_1405_6456_amd import synth

    S = synth.config(args.workload)
    ctx = lib.Context(0)
    print(json.dumps({"mode": "stencil", "workload": S.name, "nodes": S.grid.npts,
                      **stencil_streaming(ctx, S.grid.n, reps=20)}), flush=True)
    ctx.close()
    reference_copy()


def main():
    args = parse()
    if args.summarize_counters:
        return summarize_counters(*args.summarize_counters)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the solve is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    modes = {"hotpath": lambda: hotpath(args), "ground_state": lambda: ground_state(args),
             "stencil": lambda: stencil_mode(args), "counters": lambda: counters_mode(args),
             "serve": lambda: serve(args), "relax": relax_mode, "methods": methods_mode, "large": large_mode}
    modes[args.mode]()


if __name__ == "__main__":
    main()
