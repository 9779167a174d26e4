"""Benchmark of the alternating-minimisation iteration on one MI355X.

One step = one iteration of Algorithm 1 (inverse product with its FP64
refinement, positions, fused pairwise stage, linear term) over B = 1024
independent random-box problems with n = 64 agents and T = 100 instants (seeded
synthetic start/goal positions: uniform in a 10 x 10 x 5 m box, at least 1 m apart).
With `--streams S` the B problems are split into S batches on their own streams,
stepped together (one batch's pairwise stage beside the other's per-problem
kernels); the step as one batch on one stream is the default.

Prints one JSON line: pair-timestep updates/s (n(n-1)/2 * T * B per step), the
roofline of the pairwise kernel, timed with HIP events on the stream of the batch,
and the FP64 oracle timed on the host on a bounded sample (pool aggregate, and one
problem on one thread).  The pairwise kernel reads a multiplier only where its 64-row
group may hold a nonzero one and skips the rows whose agents' bounding boxes keep them
clear over its instants, so it no longer streams the multipliers: the roofline is the
vector ALU one on the dense step's arithmetic (55 FP32 flops per pair-instant, against
the 157.3 TFLOP/s FP32 peak), with the instruction-issue share and the calibrated HBM
counter bytes of the committed profile beside it, and the dense multiplier stream's
24 bytes per pair-instant as a model (its rate above the 8 TB/s peak is traffic the
kernel does not move), plus the branch census (pair-instants that take the far-pair
shortcut, multipliers rewritten).  Also in the line:
the same iteration on crowded, packed and n = 128 scenes, the structured x/y/z
solve, served p50/p99 of the serving configuration (dense BF16 product with FP64
corrections, n in 4..128, 10 / 100 / 500 requests/s) and of the structured variant,
uneven-size batching (256 problems, n in {8, 12, ..., 48}) against the same problems
solved one at a time, and the iteration time against the number of static obstacles
(16 agents).  `--serve-sweep` replaces all of this by the latency sweep over arrival rates.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3         # MI355X FP32 vector peak
SIMD_ISSUE_PER_S = 1024 * 2.4e9 / 4   # wave64 VALU instructions per second: 1 024 SIMDs, 4 cycles each
FLOPS_PER_UPDATE = 55            # FP32 flops of one dense pair-instant step (delta, s, d, projection, lambda, b_fc)
BYTES_PER_UPDATE = 24            # every FP32 multiplier read and written back, as the method states the step
READ_BYTES_PER_UPDATE = 12       # the multiplier reads alone
PROFILES = os.path.join(ROOT, "profiles")

# workloads of the pairwise stage: name -> (description, n, problems per launch, generator(n, seed))
WORKLOADS = {
    "box": ("random-box problems (uniform in 10 x 10 x 5 m, >= 1 m apart)", 64, 1024, "random_box"),
    "crowded": ("antipodal swaps through a 2 m sphere (Fibonacci lattice, +-0.05 m jitter)", 64, 1024, "swap_sphere"),
    "packed": ("starts and goals packed in a 0.2 m cube: every pair overlaps", 64, 1024, "packed_cube"),
    "box128": ("random-box problems at the n = 64 density (2:2:1 box)", 128, 256, "random_density_box"),
}


def workload_problem(name, n, seed):
    from paper_2011_04240_amd import scenarios as sc
    kind = WORKLOADS[name][3]
    if kind == "swap_sphere":
        return sc.swap_sphere(n, radius=2.0, seed=seed)
    if kind == "packed_cube":
        return sc.packed_cube(n, 0.2, seed=seed)
    return getattr(sc, kind)(n, seed=seed)


def counters_file(name, n, T, B):
    return os.path.join(PROFILES, "pairwise_%s_n%d_T%d_B%d_counters.txt" % (name, n, T, B))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=1024, help="problems per step")
    ap.add_argument("--streams", type=int, default=1,
                    help="split the problems into this many batches on their own streams (the roofline is "
                         "measured on one batch of all of them)")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--workload", default="box", choices=sorted(WORKLOADS),
                    help="scene of the timed step (box: the headline; crowded, packed: collisions common; "
                         "box128: n = 128)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the crowded, packed and n = 128 pairwise workloads")
    ap.add_argument("--T", type=int, default=100)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--solve", default="dense", choices=["dense", "structured"],
                    help="x/y/z step of the timed iteration (the structured variant is also timed beside it)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-obstacles", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=100.0)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only run the served-latency sweep over arrival rates 10..500 /s")
    ap.add_argument("--serve-precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--serve-solve", default="structured", choices=["dense", "structured"])
    ap.add_argument("--sweep-requests", type=int, default=2000,
                    help="requests per rate in the sweep (fewer where the trace would exceed 90 s)")
    ap.add_argument("--serve-chunk", type=int, default=10, help="iterations per server scheduling step")
    ap.add_argument("--serve-graphs", action="store_true",
                    help="replay the server's iterations from HIP graphs (recaptured when the resident set changes)")
    ap.add_argument("--serve-fixed-rho", action="store_true",
                    help="serve with one rho instead of the increasing schedule")
    ap.add_argument("--config-solves", action="store_true",
                    help="only time whole fixed-iteration solves of single problems of the four single-problem "
                         "configurations, on the GPU and by the oracle on the host")
    return ap.parse_args()


def kernel_source_hash():
    """Hash of the pairwise kernel's source (its block of kernels.hip, from its leading
    comment to the next kernel's) and of the shared declarations it uses."""
    csrc = os.path.join(ROOT, "paper_2011_04240_amd", "csrc")
    with open(os.path.join(csrc, "kernels.hip")) as fh:
        text = fh.read()
    a = text.index("// One workgroup per work item:")
    b = text.index("// One workgroup per problem: X = P c", a)
    h = hashlib.sha256(text[a:b].encode())
    with open(os.path.join(csrc, "common.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def counters_from_profile(path):
    """Per pairwise launch, from committed rocprofv3 counters if they were taken on the
    current kernel source: calibrated HBM bytes and wave64 VALU instructions (None where
    absent or stale)."""
    out = {"hbm_bytes_per_launch": None, "valu_insts_per_launch": None}
    if not os.path.exists(path):
        return out
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_hash():
        return out
    for k in out:
        try:
            out[k] = float(vals[k].split()[0])
        except (KeyError, ValueError, IndexError):
            pass
    return out


def _oracle_iterations(job):
    """The FP64 oracle iterating one random-box problem (seed `seed`) for about `seconds`,
    BLAS limited to one thread.  Returns (iterations, seconds).  Runs in a pool worker."""
    n, T, seconds, seed = job
    from threadpoolctl import threadpool_limits
    from oracle import am
    from paper_2011_04240_amd import scenarios as sc
    s, g = sc.random_box(n, seed=seed)
    with threadpool_limits(limits=1):
        plan = am.make_plan(n, T, 11, 10.0, 0.3, 0.6, 1.0)
        st = am.initial_state(plan, s, g)
        st = am.iterate(plan, st)                  # warm-up
        t0 = time.perf_counter()
        iters = 0
        while time.perf_counter() - t0 < seconds:
            st = am.iterate(plan, st)
            iters += 1
        dt = time.perf_counter() - t0
    return iters, dt


def _oracle_single(job):
    """The oracle's plan time (K assembly and FP64 inverse) and seconds per iteration of one
    problem with one BLAS thread: 3 warm-up iterations, then the median of 5 timed ones.
    Runs in a pool worker."""
    n, T, seed = job
    from threadpoolctl import threadpool_limits
    from oracle import am
    from paper_2011_04240_amd import scenarios as sc
    s, g = sc.random_box(n, seed=seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        plan = am.make_plan(n, T, 11, 10.0, 0.3, 0.6, 1.0)
        plan_s = time.perf_counter() - t0
        st = am.initial_state(plan, s, g)
        for _ in range(3):
            st = am.iterate(plan, st)
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            st = am.iterate(plan, st)
            times.append(time.perf_counter() - t0)
    return plan_s, float(np.median(times))


def host_description():
    """CPU model, online cores and the BLAS NumPy was built against."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        blas = "%s %s" % (blas.get("name"), blas.get("version"))
    except Exception:
        blas = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "numpy": np.__version__, "blas": blas}


def host_cores():
    """Cores this process may run on, at most 16 (the host share of one GPU)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def start_cpu_pool():
    """Worker processes for the oracle baseline, started before anything touches the GPU
    (fresh interpreters, one BLAS thread each); None if they cannot be started."""
    import multiprocessing
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    try:
        for k in saved:
            os.environ[k] = "1"
        pool = multiprocessing.get_context("spawn").Pool(host_cores())
        pool.cores = host_cores()
        return pool
    except (OSError, RuntimeError, ValueError):
        return None
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def cpu_baseline(n, T, seconds, pool=None):
    """The FP64 oracle on the host: one problem of the workload per core (seeds 0..C-1),
    all cores at once for 2 * seconds of CPU time in all (at least 2 s each), aggregate
    updates/s; in this process on one core for `seconds` without a pool."""
    npairs = n * (n - 1) // 2
    if pool is None:
        iters, dt = _oracle_iterations((n, T, seconds, 0))
        return {"value": npairs * T * iters / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
                "sample": "one n=%d T=%d random-box problem, %d FP64 iterations in %.1f s, BLAS 1 thread"
                          % (n, T, iters, dt)}
    cores = pool.cores
    plan_s, s_iter = pool.apply(_oracle_single, ((n, T, 0),))
    per = max(2.0, 2.0 * seconds / cores)
    res = pool.map(_oracle_iterations, [(n, T, per, q) for q in range(cores)], chunksize=1)
    rates = [npairs * T * it / dt for it, dt in res]
    return {"value": float(sum(rates)), "unit": "updates/s", "cores": cores, "kind": "oracle",
            "per_core": float(np.mean(rates)), "host": host_description(),
            "single_thread": {"s_per_iteration": s_iter, "updates_per_s": npairs * T / s_iter,
                              "plan_s": plan_s,
                              "method": "one n=%d T=%d random-box problem (seed 0), one BLAS thread, "
                                        "3 warm-up iterations then the median of 5" % (n, T)},
            "sample": "%d processes at once, each one n=%d T=%d random-box problem (seeds 0..%d) iterated in FP64 "
                      "for %.1f s (%d-%d iterations each), BLAS 1 thread per process"
                      % (cores, n, T, cores - 1, per, min(r[0] for r in res), max(r[0] for r in res))}


RHO_SCHEDULE = ([2.0 ** j for j in range(10)], [30 * j for j in range(10)])


def serve_trace(rate, count, precision, seed=0, max_slots=256, chunk=10, max_iters=2000, tol=1e-3,
                schedule=True, solve="structured", use_graphs=False):
    """Poisson arrivals of random-box problems (n uniform over 4..128, box at the n=64
    density) replayed in real time through the server; latency = finish - arrival.
    With `schedule`, ten increasing rho (doubling every 30 iterations, Sec. IV-A)."""
    from paper_2011_04240_amd import mato
    from paper_2011_04240_amd import scenarios as sc
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    ns = [int(x) for x in rng.integers(4, 129, size=count)]
    scen = [sc.random_density_box(n, seed=10000 * (seed + 1) + k) for k, n in enumerate(ns)]
    arr = sc.poisson_arrivals(rate, count, seed=seed)
    srv = mato.Server(T=100, n_coef=11, t_final=10.0, a=0.3, b=0.6, rho=1.0, precision=precision,
                      max_slots=max_slots, chunk=chunk, max_iters=max_iters, tol=tol,
                      rho_schedule=RHO_SCHEDULE if schedule else None, solve=solve, use_graphs=use_graphs)
    t0 = time.perf_counter()
    srv.warm(4, 128)
    warm_s = time.perf_counter() - t0
    lat, its, conv, wall = srv.run_trace(arr, [x[0] for x in scen], [x[1] for x in scen])
    srv.close()
    upd = sum(n * (n - 1) // 2 * 100 * int(k) for n, k in zip(ns, its))
    return {"rate_per_s": rate, "requests": count, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(np.mean(lat) * 1e3),
            "throughput_problems_per_s": count / wall, "updates_per_s": upd / wall,
            "converged_frac": float(np.mean(conv)), "capped_frac": float(np.mean(its >= max_iters)),
            "mean_iters": float(np.mean(its)), "wall_s": wall, "plan_warm_s": warm_s,
            "precision": precision, "solve": solve, "graphs": use_graphs, "max_slots": max_slots, "chunk": chunk, "max_iters": max_iters, "tol_m": tol,
            "rho": ({"values": RHO_SCHEDULE[0], "start_iter": RHO_SCHEDULE[1]} if schedule else 1.0)}


def serve_config5(rates=((10.0, 60), (100.0, 300), (500.0, 1000)), seed=0, max_slots=256, chunk=10,
                  max_iters=2000, tol=1e-3):
    """The serving configuration as specified: Poisson arrivals of random-box problems (n
    uniform over 4..128, box at the n = 64 density), dense x/y/z step with the inverse
    product on BF16 MFMA (three-term split, FP32 accumulation) and FP64 corrections, FP32
    state, stop at max ||f_c|| < 1e-3 m or 2000 iterations, the ten increasing rho of
    Sec. IV-A.  One server (plans for every n built beforehand) replays one trace per rate."""
    from paper_2011_04240_amd import mato
    from paper_2011_04240_amd import scenarios as sc
    srv = mato.Server(T=100, n_coef=11, t_final=10.0, a=0.3, b=0.6, rho=1.0, precision="bf16",
                      max_slots=max_slots, chunk=chunk, max_iters=max_iters, tol=tol,
                      rho_schedule=RHO_SCHEDULE, solve="dense")
    t0 = time.perf_counter()
    srv.warm(4, 128)
    warm_s = time.perf_counter() - t0
    rows = []
    for k, (rate, count) in enumerate(rates):
        rng = np.random.Generator(np.random.PCG64(5000 + k + seed))
        ns = [int(x) for x in rng.integers(4, 129, size=count)]
        scen = [sc.random_density_box(n, seed=50000 * (k + 1) + q) for q, n in enumerate(ns)]
        arr = sc.poisson_arrivals(rate, count, seed=500 + k + seed)
        lat, its, conv, wall = srv.run_trace(arr, [x[0] for x in scen], [x[1] for x in scen])
        upd = sum(n * (n - 1) // 2 * 100 * int(i) for n, i in zip(ns, its))
        rows.append({"rate_per_s": rate, "requests": count, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(np.mean(lat) * 1e3),
                     "throughput_problems_per_s": count / wall, "updates_per_s": upd / wall,
                     "converged_frac": float(np.mean(conv)), "capped_frac": float(np.mean(its >= max_iters)),
                     "mean_iters": float(np.mean(its)), "wall_s": wall})
        print(f"config-5 rate {rate}/s: p50 {rows[-1]['p50_ms']:.1f} ms, p99 {rows[-1]['p99_ms']:.1f} ms, "
              f"converged {rows[-1]['converged_frac']:.3f}", file=sys.stderr, flush=True)
    srv.close()
    return {"precision": "bf16 (three-term split) + FP64 corrections", "solve": "dense", "state": "fp32",
            "rho": {"values": RHO_SCHEDULE[0], "start_iter": RHO_SCHEDULE[1]}, "tol_m": tol,
            "max_iters": max_iters, "max_slots": max_slots, "chunk": chunk, "plan_warm_s": warm_s, "rates": rows}


def multi_stream_step(plan, starts, goals, S, tiles, steps, warmup):
    """The same B problems split into S batches, each on its own library stream, stepped
    together (graph-replayed): one batch's HBM-bound pairwise stage overlaps another's
    per-problem kernels.  Returns seconds per step of all B problems."""
    import torch
    from paper_2011_04240_amd import mato
    B = len(starts)
    parts = [list(ix) for ix in np.array_split(np.arange(B), S)]
    streams = [mato.Stream() for _ in range(S)]
    batches = [mato.Batch([plan] * len(ix), [starts[i] for i in ix], [goals[i] for i in ix], stream=st)
               for ix, st in zip(parts, streams)]
    for b in batches:
        b.set_tiles(*tiles)
        b.step(warmup, use_graph=True)
    for b in batches:
        b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in batches:
        b.step(steps, use_graph=True)
    for b in batches:
        b.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for b in batches:
        b.close()
    for st in streams:
        st.close()
    return wall / steps


def structured_step(n, T, B, starts, goals, args):
    """The same step with the structured x/y/z solve (two per-agent inverses, FP64)."""
    import torch
    from paper_2011_04240_amd import mato
    plan = mato.Plan(n, T, 11, 10.0, 0.3, 0.6, 1.0, "fp32", solve="structured")
    batch = mato.Batch([plan] * B, starts, goals)
    tiles = batch.autotune() if not args.no_autotune else batch.get_tiles()
    batch.step(args.warmup, use_graph=False)
    batch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(args.steps, use_graph=False)
    batch.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    batch.close()
    upd = n * (n - 1) // 2 * T * B
    out = {"ms_per_step": wall / args.steps * 1e3, "updates_per_s": upd * args.steps / wall, "precision": "fp32"}
    if args.streams > 1:
        sec = multi_stream_step(plan, starts, goals, args.streams, tiles, args.steps, args.warmup)
        out["streams"] = args.streams
        out["ms_per_step_streams"] = sec * 1e3
        out["updates_per_s_streams"] = upd / sec
    return out


def batch_scaling(n, T, sizes=(1, 16, 256), steps=30):
    """Updates/s of the same step at fewer problems per launch (the single-problem rate
    and partly filled GPUs), dense and structured, FP32, graph-replayed."""
    from paper_2011_04240_amd import mato
    from paper_2011_04240_amd import scenarios as sc
    npairs = n * (n - 1) // 2
    out = []
    for solve in ("dense", "structured"):
        plan = mato.Plan(n, T, 11, 10.0, 0.3, 0.6, 1.0, "fp32", solve=solve)
        for B in sizes:
            starts, goals = zip(*[sc.random_box(n, seed=q) for q in range(B)])
            b = mato.Batch([plan] * B, starts, goals)
            b.step(5)
            b.sync()
            t0 = time.perf_counter()
            b.step(steps)
            b.sync()
            dt = (time.perf_counter() - t0) / steps
            b.close()
            out.append({"solve": solve, "problems": B, "ms_per_iter": dt * 1e3,
                        "updates_per_s": npairs * T * B / dt})
        plan.close()
    return out


def solve_times(ns=(8, 16, 32), seeds=4):
    """Wall time of whole solves of one problem (batch creation, initialisation and the
    iterations until max ||f_c|| < 1e-3 m, cap 2000; plans built beforehand, as the paper
    builds its inverses offline): n agents swapping across a circle (radius max(2, n/(2 pi)) m,
    neighbours about 1 m apart) and random-box problems at the n = 64 density, ten increasing
    rho, dense and structured x/y/z step, FP32."""
    from paper_2011_04240_amd import mato
    from paper_2011_04240_amd import scenarios as sc
    rhos, starts_it = RHO_SCHEDULE
    out = []
    for solve in ("dense", "structured"):
        for n in ns:
            plans = mato.Plan.schedule(n, 100, rhos, 11, 10.0, 0.3, 0.6, "fp32", solve=solve)
            for kind in ("swap", "box"):
                times, iters = [], []
                for seed in range(seeds):
                    if kind == "swap":
                        s, g = sc.swap_circle(n, radius=max(2.0, 0.5 * n / np.pi), seed=seed)
                    else:
                        s, g = sc.random_density_box(n, seed=seed)
                    t0 = time.perf_counter()
                    b = mato.Batch([plans[0]], [s], [g])
                    b.set_rho_schedule([[p] for p in plans], starts_it)
                    b.run(2000, 1e-3, 10)
                    it, conv = b.status(0)
                    times.append(time.perf_counter() - t0)
                    iters.append(it)
                    b.close()
                out.append({"solve": solve, "n": n, "scenario": kind, "ms_median": float(np.median(times) * 1e3),
                            "iterations_median": float(np.median(iters))})
            for p in plans:
                p.close()
    return out


# single-problem configurations: label, n, T, t_final, a, b, iterations, precision, scenario
CONFIG_SOLVES = [
    ("swap circle n=4 T=50 FP64, 200 iterations", 4, 50, 5.0, 0.4, 0.8, 200, "fp64", "circle"),
    ("swap sphere n=16 T=100 FP32, 300 iterations", 16, 100, 10.0, 0.3, 0.6, 300, "fp32", "sphere"),
    ("random box n=64 T=100 FP32, 300 iterations", 64, 100, 10.0, 0.3, 0.6, 300, "fp32", "box"),
    ("random box n=64 T=100 BF16 split + FP64 correction, 300 iterations", 64, 100, 10.0, 0.3, 0.6, 300, "bf16",
     "box"),
]


def _config_scenario(kind, n, seed):
    from paper_2011_04240_amd import scenarios as sc
    if kind == "circle":
        return sc.swap_circle(n, seed=seed)
    if kind == "sphere":
        return sc.swap_sphere(n, seed=seed)
    return sc.random_box(n, seed=seed)


def _oracle_config_solve(job):
    """Plan and whole fixed-iteration solves of one configuration by the FP64 oracle, one
    BLAS thread (pool worker): plan seconds and the median of `runs` solves after `warm`."""
    n, T, tf, a, b, iters, kind, warm, runs = job
    from threadpoolctl import threadpool_limits
    from oracle import am
    s, g = _config_scenario(kind, n, 0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        plan = am.make_plan(n, T, 11, tf, a, b, 1.0)
        plan_s = time.perf_counter() - t0
        times = []
        for k in range(warm + runs):
            t0 = time.perf_counter()
            am.solve(plan, s, g, iters)
            if k >= warm:
                times.append(time.perf_counter() - t0)
    return plan_s, float(np.median(times))


def config_solves(pool):
    """Whole fixed-iteration solves of single problems of the specified configurations, on
    the GPU (batch of one: creation, initialisation, iterations, coefficients back; plan
    built beforehand and timed apart; one warm-up, median of 5) and by the FP64 oracle on
    the host (one BLAS thread per process, the configurations in parallel)."""
    from paper_2011_04240_amd import mato
    jobs = [(n, T, tf, a, b, it, kind, 1 if n >= 64 else 3, 3 if n >= 64 else 5)
            for _, n, T, tf, a, b, it, _, kind in CONFIG_SOLVES]
    cpu = pool.map_async(_oracle_config_solve, jobs, chunksize=1) if pool is not None else None
    out = []
    for label, n, T, tf, a, b, iters, prec, kind in CONFIG_SOLVES:
        s, g = _config_scenario(kind, n, 0)
        t0 = time.perf_counter()
        plan = mato.Plan(n, T, 11, tf, a, b, 1.0, prec)
        plan_s = time.perf_counter() - t0
        times = []
        for k in range(6):
            t0 = time.perf_counter()
            bt = mato.Batch([plan], [s], [g])
            bt.run(iters, 0.0, iters)
            bt.coeffs(0)
            times.append(time.perf_counter() - t0)
            bt.close()
        plan.close()
        gpu_s = float(np.median(times[1:]))
        upd = n * (n - 1) // 2 * T * iters
        out.append({"config": label, "gpu_plan_s": plan_s, "gpu_solve_s": gpu_s, "gpu_updates_per_s": upd / gpu_s})
        print(f"{label}: GPU {gpu_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    if cpu is not None:
        for row, job, (plan_s, sec) in zip(out, jobs, cpu.get()):
            n, T, iters = job[0], job[1], job[5]
            row.update({"oracle_plan_s": plan_s, "oracle_solve_s": sec,
                        "oracle_updates_per_s": n * (n - 1) // 2 * T * iters / sec,
                        "oracle_s_per_iteration": sec / iters, "speedup": sec / row["gpu_solve_s"]})
    return out


def obstacle_scaling(n=16, counts=(0, 8, 16, 32, 64, 128), batch=256, iters=30):
    """Iteration time against the number of static obstacles (16 agents, T = 100): one
    problem alone and `batch` problems per launch; structured solve, FP32, graphs."""
    from paper_2011_04240_amd import mato
    from paper_2011_04240_amd import scenarios as sc
    out = []
    for k in counts:
        scen = [sc.obstacle_box(n, k, seed=30000 + q) for q in range(batch)]
        plan = mato.Plan(n, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32", solve="structured", n_obs=k)
        row = {"n_obs": k, "rows": n * (n - 1) // 2 + n * k}
        for label, m in (("single", 1), ("batch", batch)):
            b = mato.Batch([plan] * m, [x[0] for x in scen[:m]], [x[1] for x in scen[:m]],
                           obstacles_list=[x[2] for x in scen[:m]])
            b.step(3)
            b.sync()
            t0 = time.perf_counter()
            b.step(iters)
            b.sync()
            dt = (time.perf_counter() - t0) / iters
            b.close()
            row[label + "_ms_per_iter"] = dt * 1e3
            row[label + "_row_updates_per_s"] = row["rows"] * 100 * m / dt
        out.append(row)
    return {"agents": n, "T": 100, "problems_per_launch": batch, "solve": "structured", "precision": "fp32",
            "points": out}


def mixed_batching(count=256, iters=30, seed=0):
    """Uneven sizes in one launch per stage (graph-replayed, autotuned tiles) against the
    plain per-problem method (each problem alone, separate launches, no graphs)."""
    from paper_2011_04240_amd import mato
    from paper_2011_04240_amd import scenarios as sc
    ns = sc.agent_counts(count, list(range(8, 49, 4)), seed=seed)
    scen = [sc.random_box(n, seed=20000 + k) for k, n in enumerate(ns)]
    plans = {n: mato.Plan(n, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32") for n in sorted(set(ns))}
    batch = mato.Batch([plans[n] for n in ns], [x[0] for x in scen], [x[1] for x in scen])
    tiles = batch.autotune()
    batch.step(3)
    batch.sync()
    t0 = time.perf_counter()
    batch.step(iters, use_graph=True)
    batch.sync()
    t_batch = time.perf_counter() - t0
    batch.close()
    splans = {n: mato.Plan(n, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32", solve="structured") for n in sorted(set(ns))}
    sbatch = mato.Batch([splans[n] for n in ns], [x[0] for x in scen], [x[1] for x in scen])
    sbatch.set_tiles(*tiles)
    sbatch.step(3)
    sbatch.sync()
    t0 = time.perf_counter()
    sbatch.step(iters, use_graph=True)
    sbatch.sync()
    t_struct = time.perf_counter() - t0
    sbatch.close()
    solo = [mato.Batch([plans[n]], [scen[k][0]], [scen[k][1]]) for k, n in enumerate(ns)]
    for b in solo:
        b.step(1, use_graph=False)
    for b in solo:
        b.sync()
    t0 = time.perf_counter()
    for b in solo:
        b.step(iters, use_graph=False)
        b.sync()
    t_solo = time.perf_counter() - t0
    upd = sum(n * (n - 1) // 2 * 100 for n in ns) * iters
    return {"problems": count, "n_values": sorted(set(ns)), "iterations_timed": iters,
            "batched": {"ms_per_iter": t_batch / iters * 1e3, "updates_per_s": upd / t_batch,
                        "problems_per_s_300_iters": count / (t_batch / iters * 300),
                        "tiles": {"items_per_wg": tiles[0], "threads": tiles[1]}},
            "batched_structured": {"ms_per_iter": t_struct / iters * 1e3, "updates_per_s": upd / t_struct,
                                   "problems_per_s_300_iters": count / (t_struct / iters * 300)},
            "per_problem": {"ms_per_iter_all": t_solo / iters * 1e3, "updates_per_s": upd / t_solo,
                            "problems_per_s_300_iters": count / (t_solo / iters * 300)},
            "speedup": t_solo / t_batch}


def stream_ceiling(nbytes, probe="copy"):
    """Best rate of the library's streaming copy, its in-place streaming update (equal HBM
    reads and writes at the same addresses) or its streaming read, over a few grid sizes, for
    `nbytes` read (and as many written by the copy and the update): the practical ceilings of
    the multiplier stream."""
    from paper_2011_04240_amd import mato
    fn = {"copy": mato.mato_stream_copy, "update": mato.mato_stream_update, "read": mato.mato_stream_read}[probe]
    moved = 1 if probe == "read" else 2
    nbytes -= nbytes % 16
    best = None
    for grid in (1024, 2048, 4096, 16384, 65536):
        ms = fn(nbytes, grid, 10)
        gbs = moved * nbytes / (ms * 1e-3) / 1e9
        if best is None or gbs > best[0]:
            best = (gbs, grid, ms)
    return {"GBps": best[0], "grid": best[1], "ms_per_pass": best[2], "bytes_each_way": nbytes}


def copy_calibration(mib):
    import torch
    x = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": mib * (1 << 20), "launches": 3}))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the problems are independent and the library "
              "has no multi-GPU path; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.serve_sweep:
        sweep = []
        for k, r in enumerate([10, 20, 50, 100, 200, 500]):
            sweep.append(serve_trace(r, min(args.sweep_requests, int(r * 90)), args.serve_precision, seed=k,
                                     chunk=args.serve_chunk, schedule=not args.serve_fixed_rho,
                                     solve=args.serve_solve, use_graphs=args.serve_graphs))
            print(f"rate {r}/s: p50 {sweep[-1]['p50_ms']:.1f} ms, p99 {sweep[-1]['p99_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
        print(json.dumps({"metric": "served p50/p99 solve latency", "unit": "ms", "sweep": sweep,
                          "data": "synthetic", "n_gpus": 1}))
        return
    pool = None if args.no_cpu_baseline else start_cpu_pool()     # before the GPU is initialised
    try:
        if args.config_solves:
            import torch
            torch.cuda.set_device(0)
            print(json.dumps({"metric": "whole solve seconds of single problems", "data": "synthetic", "n_gpus": 1,
                              "oracle_cores": pool.cores if pool is not None else 0,
                              "configs": config_solves(pool)}))
            return
        run_main(args, pool)
    finally:
        if pool is not None:
            pool.terminate()
            pool.join()


def branch_census(batch, problems, n):
    """One more iteration of `problems` of the batch, observed through the state hooks: the
    share of pair-instants that take the pairwise stage's far-pair shortcut (every axis of
    the multiplier +0 before the step and s^2 > 1.0001 at the step's positions, the test
    the kernel makes, here in FP64 from the FP32 positions), and the share of multiplier elements whose bits the step changed
    (the only ones it writes back)."""
    iu, ju = np.triu_indices(n, 1)
    before = [batch.get_state(q)["lam"] for q in problems]
    batch.step(1, use_graph=False)
    batch.sync()
    short = changed = total = 0
    for q, lam0 in zip(problems, before):
        st = batch.get_state(q, X=True)
        X = st["X"].astype(np.float64)                # [n][3][T]: the positions of this step
        d = X[iu] - X[ju]
        s2 = (d[:, 0] ** 2 + d[:, 1] ** 2) / 0.3 ** 2 + d[:, 2] ** 2 / 0.6 ** 2   # [pair][T]
        zero = np.all(lam0.view(np.uint32) == 0, axis=-1)
        short += int(np.count_nonzero(zero & (s2 > 1.0001)))
        changed += int(np.count_nonzero(lam0.view(np.uint32) != st["lam"].view(np.uint32)))
        total += zero.size
    return {"shortcut_frac": short / total, "general_frac": 1.0 - short / total,
            "written_frac": changed / (3 * total), "sampled_problems": len(problems)}


def time_workload(name, T, steps, warmup, precision, solve, autotune=True, warm_iters=None):
    """Iterations of B problems of one workload in one batch (eager launches, HIP events
    around every kernel on the batch's stream): seconds per step, the pairwise kernel's
    average launch, the branch census after the timed steps and the roofline of the
    pairwise kernel (vector ALU on the dense step's 55 flops per pair-instant; the dense
    multiplier stream's 24 bytes per pair-instant as a model)."""
    import torch
    from paper_2011_04240_amd import mato
    desc, n, B, _ = WORKLOADS[name]
    npairs = n * (n - 1) // 2
    starts, goals = zip(*[workload_problem(name, n, q) for q in range(B)])
    t0 = time.perf_counter()
    plan = mato.Plan(n, T, 11, 10.0, 0.3, 0.6, 1.0, precision, solve=solve)
    plan_s = time.perf_counter() - t0
    batch = mato.Batch([plan] * B, starts, goals)
    tiles = batch.autotune() if autotune else batch.get_tiles()
    batch.step(warmup if warm_iters is None else warm_iters, use_graph=False)
    batch.sync()
    batch.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps, use_graph=False)
    batch.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms, pw_ms, launches = batch.last_times()
    batch.timing(False)
    pw_avg_s = pw_ms / max(launches, 1) / 1e3
    units = npairs * T * B
    r_max, _, _ = batch.residuals(0)
    census = branch_census(batch, list(range(min(8, B))), n)
    batch.close()
    plan.close()
    achieved = FLOPS_PER_UPDATE * units / pw_avg_s / 1e12
    prof = counters_from_profile(counters_file(name, n, T, B))
    traffic = prof["hbm_bytes_per_launch"]
    dense_GBps = BYTES_PER_UPDATE * units / pw_avg_s / 1e9
    roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
            "kernel": "pairwise_fx_kernel" if precision != "fp64" else "pairwise_kernel",
            "avg_launch_ms": pw_avg_s * 1e3,
            "flops_per_unit": FLOPS_PER_UPDATE, "algorithmic_flops_per_launch": FLOPS_PER_UPDATE * units,
            "units_per_launch": units,
            "hbm_model": {"bytes_per_unit": BYTES_PER_UPDATE,
                          "algorithmic_bytes_per_launch": BYTES_PER_UPDATE * units,
                          "achieved_GBps": dense_GBps, "frac_of_peak": dense_GBps / HBM_PEAK_GBS},
            "shortcut_frac": census["shortcut_frac"], "written_frac": census["written_frac"]}
    if traffic is not None:
        roof["traffic_GBps"] = traffic / pw_avg_s / 1e9
        roof["traffic_frac"] = roof["traffic_GBps"] / HBM_PEAK_GBS
    if prof["valu_insts_per_launch"] is not None:
        roof["valu_insts_per_launch"] = prof["valu_insts_per_launch"]
        roof["valu_issue_frac"] = prof["valu_insts_per_launch"] / SIMD_ISSUE_PER_S / pw_avg_s
    return {"workload": desc, "name": name, "n": n, "T": T, "problems": B, "precision": precision, "solve": solve,
            "ms_per_step": wall / steps * 1e3, "updates_per_s": units * steps / wall,
            "device_ms_per_step": total_ms / steps, "plan_s": plan_s,
            "tiles": {"items_per_wg": tiles[0], "threads": tiles[1]}, "census": census, "roofline": roof,
            "final_r_max_problem0": float(r_max[-1]) if len(r_max) else None}


def run_main(args, pool):
    import torch
    from paper_2011_04240_amd import mato

    n, T, B = args.n, args.T, args.batch
    npairs = n * (n - 1) // 2
    torch.cuda.set_device(0)
    name = args.workload
    if (WORKLOADS[name][1], WORKLOADS[name][2]) != (n, B):
        WORKLOADS[name] = (WORKLOADS[name][0], n, B, WORKLOADS[name][3])
    head = time_workload(name, T, args.steps, args.warmup, args.precision, args.solve,
                         autotune=not args.no_autotune)
    roof = head["roofline"]
    units = npairs * T * B
    read_bytes = READ_BYTES_PER_UPDATE * units
    stream_rd = stream_ceiling(read_bytes, "read")
    stream = stream_ceiling(read_bytes)
    stream_upd = stream_ceiling(read_bytes, "update")
    # the streaming probes over the dense multiplier array: the rate a multiplier stream
    # would reach (context for the model; the kernel reads only flagged groups)
    roof["hbm_model"].update({"stream_read": stream_rd, "stream_copy": stream, "stream_update": stream_upd,
                              "read_bytes_per_launch": read_bytes,
                              "read_GBps": read_bytes / (roof["avg_launch_ms"] * 1e-3) / 1e9})
    roof["hbm_model"]["read_frac_of_stream_read"] = roof["hbm_model"]["read_GBps"] / stream_rd["GBps"]
    if roof["traffic"] is not None:
        roof["traffic_frac_of_stream_read"] = roof["traffic_GBps"] / stream_rd["GBps"]
    single = {"ms_per_step": head["ms_per_step"], "updates_per_s": head["updates_per_s"]}
    value, ms_per_step = head["updates_per_s"], head["ms_per_step"]
    if args.streams > 1:
        starts, goals = zip(*[workload_problem(name, n, q) for q in range(B)])
        plan = mato.Plan(n, T, 11, 10.0, 0.3, 0.6, 1.0, args.precision, solve=args.solve)
        sec = multi_stream_step(plan, starts, goals, args.streams, (head["tiles"]["items_per_wg"],
                                head["tiles"]["threads"]), args.steps, args.warmup)
        plan.close()
        value = units / sec
        ms_per_step = sec * 1e3
    out = {
        "metric": "pair-timestep updates/s at n=64,T=100",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s, n=%d agents, T=%d instants, %d problems per launch" % (head["workload"], n, T, B),
                   "n": n, "T": T, "problems": B, "precision": args.precision, "solve": args.solve,
                   "streams": args.streams, "tiles": head["tiles"],
                   "device_ms_per_step": head["device_ms_per_step"], "plan_s": head["plan_s"]},
        "roofline": roof,
        "census": head["census"],
        "final_r_max_problem0": head["final_r_max_problem0"],
        "single_stream": single,
    }
    if args.solve == "dense":
        starts, goals = zip(*[workload_problem(name, n, q) for q in range(B)])
        out["structured_step"] = structured_step(n, T, B, starts, goals, args)
    if not args.no_workloads:
        # the pairwise stage where collisions are common (its general branch) and at the
        # largest agent count of the serving configuration; warmed 30 iterations
        out["workloads"] = [time_workload(w, T, args.steps, 30, args.precision, args.solve,
                                          autotune=not args.no_autotune)
                            for w in ("crowded", "packed", "box128") if w != name]
    if not args.no_mixed:
        out["batch_scaling"] = batch_scaling(n, T)
    if not args.no_serve:
        out["served"] = serve_trace(args.serve_rate, args.serve_requests, args.serve_precision,
                                    chunk=args.serve_chunk, schedule=not args.serve_fixed_rho,
                                    solve=args.serve_solve, use_graphs=args.serve_graphs)
        out["served"]["variant"] = "structured x/y/z step in FP64 (not the configuration's dense BF16 product)"
    if not args.no_serve:
        out["served_config5"] = serve_config5()
    if not args.no_mixed:
        out["mixed_batching"] = mixed_batching()
    if not args.no_obstacles:
        out["obstacle_scaling"] = obstacle_scaling()
    if not args.no_mixed:
        out["solve_times"] = solve_times()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, T, args.cpu_seconds, pool)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
