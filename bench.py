"""Benchmark: eigenpairs/s of full solves (Algorithm 3.2 + corrections to a
1e-8 relative residual) on one MI355X, with the dominant kernel's HBM roofline
and the CPU oracle timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1] [--precision mixed|fp64]
    python bench.py --config 4 [--requests R] [--rate HZ] [--n-hi N]     (serving stream)

A step is one whole solve of the workload: nested start from the coarsest
level, then finest-level corrections until max_{j<=q} rho_j <= 1e-8.  Inputs
(the hierarchy) are resident in HBM before the timed region starts.
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Per-workload solver options (coarse size and block width: the paper's two
# improvement strategies, Section 4.5)
WORKLOADS = {
    0: dict(name="unit square P1, 31x31 interior (N=961), q=4", coarse_max=130, qe=4),
    1: dict(name="jittered L-shape P1, h=1/256 (N=195585), q=10", coarse_max=512, qe=16),
    2: dict(name="3D checkerboard cube P1, 100^3 cells (N=970299), q=20", coarse_max=512, qe=32),
    3: dict(name="oscillator -Lap+r^2 on (-6,6)^2, 2047^2 interior (N=4190209), q=64", coarse_max=700, qe=68),
}


def cpu_baseline(idx, qe, coarse_max, tol):
    """The oracle (plain FP64 CPU, its own setup and Gauss-Seidel V-cycle) timed
    on one full solve of the same workload, setup excluded, one thread."""
    code = r"""
import json, sys, time
sys.path.insert(0, %r)
from workloads import configs
from oracle import Oracle, amg
p = configs.config(%d)
A = amg.csr(p["rowptr"], p["col"], p["A"], p["n"])
M = amg.csr(p["rowptr"], p["col"], p["M"], p["n"])
o = Oracle(A, M, q=p["q"], qe=%d, coarse_max=%d, coarse_min=2 * %d + 2, smoother="gs")
t = time.perf_counter()
lam, U, info = o.solve(tol=%r, max_steps=400)
dt = time.perf_counter() - t
print(json.dumps({"seconds": dt, "steps": info["steps"], "q": p["q"], "conv": bool(info["rho"][:p["q"]].max() <= %r)}))
""" % (ROOT, idx, qe, coarse_max, qe, tol, tol)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": d["q"] / d["seconds"], "unit": "eigenpairs/s", "cores": 1, "kind": "oracle",
            "sample": "one full oracle solve of the same workload (nested start, Gauss-Seidel V(1,1), "
                      "%d corrections to rho<=%g, %.1f s), setup excluded, 1 thread" % (d["steps"], tol, d["seconds"])}


def serving(args):
    """Serving stream: seeded requests from the three mesh families with uneven N
    and q, Poisson arrivals at a fixed rate, admission by device footprint and
    continuous batching over a stream pool (mixed precision).  Beside it, the
    same requests solved one after another as plain single-instance solves, in
    FP64 and in mixed precision.  Host setup (the AMG hierarchy) is done before
    each timed pass; binding (device workspace) and the solve are inside."""
    import torch
    import paper_1503_08462_amd as ae
    from paper_1503_08462_amd.serving import Server
    from workloads import configs

    reqs = configs.request_stream(args.requests, seed=5, n_lo=10_000, n_hi=args.n_hi)
    probs = [configs.build_request(r) for r in reqs]
    qs = np.array([p["q"] for p in probs])
    gaps = -np.log1p(-np.array([r["u_arrival"] for r in reqs])) / args.rate
    arrivals = np.cumsum(gaps) - gaps[0]
    tol = args.tol

    def contexts(prec):
        return [ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"],
                           ae.defaults(coarse_max=512, qe=p["qe"], precision=prec, tol=tol,
                                       use_graph=args.serve_graph if prec == ae.PREC_MIXED else 0)) for p in probs]

    def solo(prec):
        cs = contexts(prec)
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        t = time.perf_counter()
        lat, bad = [], []
        for k, c in enumerate(cs):
            t1 = time.perf_counter()
            c.bind(stream=stream)
            c.init(ae.INIT_NESTED)
            _, ok = c.solve(tol, 400)
            if not ok:
                bad.append(k)
            c.close()
            c.workspace = None
            lat.append(time.perf_counter() - t1)
        torch.cuda.synchronize()
        if bad:
            raise SystemExit("solo solves of requests %s did not converge" % bad)
        return qs.sum() / (time.perf_counter() - t), lat

    # warm-up: one request end to end
    c = contexts(ae.PREC_MIXED)[0]
    c.bind()
    c.init(ae.INIT_NESTED)
    c.solve(tol, 400)
    c.close()
    del c
    solo64, _ = solo(ae.PREC_FP64)
    solo32, _ = solo(ae.PREC_MIXED)

    cs = contexts(ae.PREC_MIXED)
    fps = sorted(c.footprint() for c in cs)
    budget = int(args.budget_gb * 2 ** 30)
    srv = Server(max(budget, fps[-1]), n_streams=args.streams, steps_per_round=args.steps_per_round,
                 max_active=args.max_active if args.max_active > 0 else None,
                 context_factory=lambda p, o: cs[p["_k"]],
                 batch_fn=None if args.joint else (lambda cs_, steps: ae.correct_batch(cs_, steps)),
                 init_fn=(lambda cs_: ae.init_batch_joint(cs_)) if args.joint_init else None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while i < len(probs) or srv.queue or srv.active:
        now = time.perf_counter() - t0
        while i < len(probs) and arrivals[i] <= now:
            srv.submit(dict(probs[i], _k=i), tol=tol, max_steps=400, arrival=t0 + arrivals[i])
            i += 1
        if srv.queue or srv.active:
            srv.round()
        elif i < len(probs):
            time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    res = srv.results()
    bad = [k for k, r in res.items() if not r["converged"]]
    if bad:
        raise SystemExit("served requests %s did not converge" % bad)
    lat = srv.latency()
    served = qs.sum() / makespan
    ns = [p["n"] for p in probs]
    out = {
        "metric": "eigenpairs/sec to 1e-8 rel. residual (served stream)",
        "value": served,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": makespan * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serving stream: %d seeded requests (L-shape, checkerboard cube, oscillator), "
                               "N in [%d, %d], q in {4, 8, 16, 32}, Poisson arrivals at %g/s"
                               % (len(probs), min(ns), max(ns), args.rate),
                   "requests": len(probs), "eigenpairs": int(qs.sum()), "budget_gb": args.budget_gb,
                   "streams": args.streams, "steps_per_round": args.steps_per_round, "tol": tol,
                   "max_active": args.max_active or None,
                   "graph_steps": bool(args.serve_graph), "joint_small_solves": bool(args.joint),
                   "joint_starts": bool(args.joint_init)},
        "p50_ms": lat["p50_s"] * 1e3,
        "p99_ms": lat["p99_s"] * 1e3,
        "peak_resident_gb": srv.peak_in_use / 2 ** 30,
        "rounds": srv.rounds,
        "solo_fp64_eigenpairs_per_s": solo64,
        "solo_mixed_eigenpairs_per_s": solo32,
        "served_vs_solo_fp64": served / solo64,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def load_traffic(kernel, workload_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if any."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (kernel, workload_tag))
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            return float(line.split(":", 1)[1])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--coarse-max", type=int, default=0, help="override the workload's coarsest-level bound")
    ap.add_argument("--qe", type=int, default=0, help="override the workload's block width")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=1,
                    help="replay captured correction steps (the second step of each chunk of three or more runs "
                         "eagerly and carries the per-kernel event timing)")
    ap.add_argument("--tune", type=int, default=1,
                    help="choose the row kernels' columns per lane by timing (on-disk cache) before the timed region")
    ap.add_argument("--smoother", default="chebyshev", choices=["l1jacobi", "chebyshev"])
    ap.add_argument("--requests", type=int, default=24, help="serving stream (config 4): number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serving stream: Poisson arrival rate, 1/s")
    ap.add_argument("--n-hi", type=int, default=150_000, help="serving stream: largest N drawn")
    ap.add_argument("--budget-gb", type=float, default=8.0, help="serving stream: device memory budget")
    ap.add_argument("--streams", type=int, default=8, help="serving stream: stream pool size")
    ap.add_argument("--steps-per-round", type=int, default=2, help="serving stream: corrections per round")
    ap.add_argument("--serve-graph", type=int, default=1, help="serving stream: replay captured steps (or, with "
                                                                "--joint, each request's own parts of a step)")
    ap.add_argument("--max-active", type=int, default=0, help="serving stream: requests on the device at once "
                                                                 "(0: the memory budget alone decides)")
    ap.add_argument("--joint", type=int, default=1, help="serving stream: solve the members' small eigenproblems "
                                                         "in shared launches")
    ap.add_argument("--joint-init", type=int, default=0, help="serving stream: start the requests admitted in a "
                                                              "round together (init_batch_joint)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run one plain 256 MiB device copy whose HBM counters "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus)
        sys.exit(2)

    if args.config == 4:
        serving(args)
        return

    import torch
    import paper_1503_08462_amd as ae
    from workloads import configs

    wl = dict(WORKLOADS[args.config])
    if args.coarse_max:
        wl["coarse_max"] = args.coarse_max
    if args.qe:
        wl["qe"] = args.qe
    p = configs.config(args.config)
    prec = ae.PREC_MIXED if args.precision == "mixed" else ae.PREC_FP64
    t0 = time.perf_counter()
    smoother = ae.SMOOTH_CHEBYSHEV if args.smoother == "chebyshev" else ae.SMOOTH_L1JACOBI
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"],
                     ae.defaults(coarse_max=wl["coarse_max"], qe=wl["qe"], precision=prec, use_graph=args.graph,
                                 smoother=smoother, cheb_degree=2, cheb_lo=0.25))
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    ctx.bind(stream=stream)
    info = ctx.info()
    tuning = None
    if args.tune:
        from paper_1503_08462_amd import autotune
        t1 = time.perf_counter()
        rep = autotune.tune(ctx)
        tuning = {"seconds": round(time.perf_counter() - t1, 3),
                  "cpt": {"%s@%d" % (v["kind"], v["level"]): v["cpt"] for v in rep.values()}}
    for _ in range(args.warmup):
        ctx.init(ae.INIT_NESTED)
        ctx.solve(args.tol, 400)
    ctx.timing(True)
    lat, steps = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        ctx.init(ae.INIT_NESTED)
        lam, ok = ctx.solve(args.tol, 400)
        lat.append(time.perf_counter() - t)
        pr = ctx.progress()
        if not ok:
            raise SystemExit("solve did not converge: %s" % pr)
        steps.append(pr["steps"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    stats = ctx.site_stats()
    ctx.timing(False)
    if args.copy_calibration:
        n = 32 << 20  # 256 MiB of doubles read, 256 MiB written
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    q = p["q"]
    sites = {}
    for name, (amount, ms, n) in stats.items():
        if n == 0:
            continue
        avg = ms / n * 1e-3
        if name == "gram":
            sites[name] = {"avg_us": avg * 1e6, "launches": n, "tflops": amount / avg / 1e12}
        elif name == "small":
            sites[name] = {"avg_us": avg * 1e6, "launches": n}
        else:
            sites[name] = {"avg_us": avg * 1e6, "launches": n, "gbs": amount / avg / 1e9}
    # the roofline line covers the streaming kernel with the largest total time
    # on the finest level; the small coarse-space kernels (one workgroup per
    # eigenvalue, latency-bound) are reported beside it
    hbm_sites = [s for s in sites if s not in ("gram", "small")]
    dom = max(hbm_sites, key=lambda s: stats[s][1]) if hbm_sites else None
    roofline = None
    if dom:
        amount, ms, n = stats[dom]
        achieved = amount / (ms / n * 1e-3) / 1e9
        cheb = args.smoother == "chebyshev"
        kernel_name = {"residual": "k_residual", "presmooth": "k_cheb_pre" if cheb else "k_smooth_pre",
                       "postsmooth": "k_cheb_post2" if cheb else "k_smooth_post",
                       "dualspmm": "k_dual_spmm", "restrict": "k_spmm",
                       "final": "k_final" if wl["qe"] > 32 else "k_final_rows"}[dom]
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": load_traffic(kernel_name, "config%d_%s" % (args.config, args.precision)),
                    "kernel": kernel_name, "site": dom, "alg_bytes_per_launch": amount,
                    "avg_launch_us": round(ms / n * 1e3, 2)}
    small = None
    if "small" in sites:
        tot = sum(v[1] for k, v in stats.items() if v[2] > 0)
        small = {"bound": "latency", "avg_us_per_step": round(sites["small"]["avg_us"], 1),
                 "share_of_timed_sites": round(stats["small"][1] / tot, 3) if tot > 0 else None}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config, wl["qe"], wl["coarse_max"], args.tol)
    out = {
        "metric": "eigenpairs/sec to 1e-8 rel. residual",
        "value": q * args.steps / elapsed,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == ae.PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "N": int(p["n"]), "q": q, "qe": info["qe"],
                   "levels": info["dims"].tolist(), "precision": args.precision, "tol": args.tol,
                   "smoother": ("l1-jacobi" if args.smoother == "l1jacobi" else "chebyshev degree 2 on [0.25, 1]")
                               + " V(1,1)", "start": "nested (Algorithm 3.2)",
                   "steps_launch": ("captured hipGraph replays; the second step of each enqueued chunk of three "
                                    "or more eager and event-timed" if args.graph else "eager")},
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "corrections_per_solve": float(np.mean(steps)),
        "setup_s": setup_s,
        "tuning": tuning,
        "roofline": roofline,
        "small_solver": small,
        "sites": sites,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
