"""Benchmark of the direct factor-and-solve of the root-coupled branch system.

One step = the whole hot path on one system held in HBM: Algorithm 1 (tail factor,
coupling solve, Schur update, FP64 root reduction and root Cholesky) followed by
Algorithm 2 (two-level triangular solves) -- for the headline path in FP32 with one
FP64-residual refinement correction, and alongside it the plain FP64 path.  The
workload is the metric configuration S=512 scenarios, N=256 stages, n=32 (synthetic
seeded inputs; the paper's quadrotor systems are not available).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_MFMA_PEAK_TFS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ir-steps", type=int, default=1)
    ap.add_argument("--window-depth", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (accuracy + CPU baseline)")
    ap.add_argument("--separate", action="store_true",
                    help="time separate factor and solve calls (default: the forward "
                         "substitution of the first solve runs inside the factorization)")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--systems", type=int, default=1024,
                    help="batching workload (--config c4): number of systems")
    ap.add_argument("--tune", action="store_true",
                    help="batching workload: autotune the launch configuration per shape class")
    ap.add_argument("--no-graph", action="store_true",
                    help="batching workload: launch eagerly instead of replaying a HIP graph")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (counter calibration "
                         "for the HBM traffic figures) and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The translation unit of the factor pass kernels: the measured HBM traffic of a
# factor pass stays valid while none of these files changes.
FACTOR_SOURCES = ("factor.hip", "bmpc_internal.h", "blockops.h", "multi.h", "regblock.h")


def source_digest(names=None):
    """Digest of the code of the named files under csrc/ (all of them by default):
    line comments, trailing blanks and empty lines do not count, so that a comment edit
    does not retire counters taken on the same code."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_29977_amd", "csrc")
    for name in sorted(names if names is not None else os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            code = [ln.split("//", 1)[0].rstrip() for ln in f]
        h.update(name.encode())
        h.update("\n".join(ln for ln in code if ln).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class, digest):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/traffic.json),
    used only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_class)
    if not ent or ent.get("source_digest") != digest:
        return None
    return ent.get("bytes_per_launch")


def bench_hetero(args):
    """Batching workload: independent systems with S ~ U[8, 256], N ~ U[16, 256],
    n ~ {8, 16, 32}, delta log-uniform in [1e-4, 1], one right-hand side, FP32 + one
    refinement correction, all in one ragged plan (every step one launch over all
    systems, nothing padded), replayed from a HIP graph.  One step solves every system
    once (factor + refined solve)."""
    import numpy as np
    import torch

    from paper_2609_29977_amd import bmpc
    from synth.branch_system_gpu import make_system_gpu

    K = args.systems
    rng = np.random.default_rng(args.seed)
    shapes, deltas = [], []
    for _ in range(K):
        S = int(rng.integers(8, 257))
        N = int(rng.integers(16, 257))
        n = int(rng.choice([8, 16, 32]))
        shapes.append((S, N, n, 1))
        deltas.append(float(10 ** rng.uniform(-4, 0)))
    # Autotuned mapping: one bmpc_autotune run per shape class (block size x stage
    # range), timed on a batch of the class's mean shape with as many systems as the
    # class holds (capped at 16 GB of input), so that the tuner sees the class at the
    # load it runs under; its choice goes to every system of the class.
    tuned = {}
    options = None
    if args.tune:
        t0 = time.perf_counter()
        classes = [(n, lo, hi) for n in (8, 16, 32) for lo, hi in ((16, 64), (65, 128), (129, 256))]
        for n, lo, hi in classes:
            members = [(S, N) for S, N, nn, _ in shapes if nn == n and lo <= N <= hi]
            if not members:
                continue
            S_m = int(round(np.mean([m[0] for m in members])))
            N_m = int(round(np.mean([m[1] for m in members])))
            per_sys = S_m * (2 * N_m + 1) * n * n * 8
            B = max(1, min(len(members), int(16e9 // per_sys)))
            wd, flags, ms, cand = bmpc.autotune(S_m, N_m, n, 1, "fp32", reps=3, num_systems=B)
            tuned[f"n={n} N={lo}..{hi}"] = {"window_depth": wd, "flags": flags,
                                           "tuned_on": {"S": S_m, "N": N_m, "systems": B},
                                           "best_ms": round(ms, 4),
                                           "candidate_ms": [round(c, 4) for c in cand]}
        def cls(n, N):
            return next(v for k, v in tuned.items() if k.startswith(f"n={n} ") and
                        int(k.split("N=")[1].split("..")[0]) <= N <= int(k.split("..")[1]))
        options = [(cls(n, N)["window_depth"], cls(n, N)["flags"]) for S, N, n, _ in shapes]
        log(f"autotuned {len(tuned)} shape classes in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    side = torch.cuda.Stream()
    rp = bmpc.RaggedPlan(shapes, "fp32", stream=side, options=options)
    analyze_s = time.perf_counter() - t0
    sz = rp.sizes
    f64 = torch.float64
    D, E, C, R = (torch.empty(max(k, 1), dtype=f64, device="cuda") for k in sz[:4])
    b = torch.empty(sz[4], dtype=f64, device="cuda")
    x = torch.zeros_like(b)
    for i, (S, N, n, _) in enumerate(shapes):
        for which, (dst, t) in enumerate(zip((D, E, C, R, b),
                                             make_system_gpu(S, N, n, 1, deltas[i], 1000 + i))):
            if t.numel():
                rp.unpack(which, dst, i).copy_(t.reshape(-1))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"{K} systems in one ragged plan, analysed in {analyze_s:.1f}s, set up in "
        f"{time.perf_counter() - t0:.1f}s; inputs {sum(sz) * 8 / 1e9:.1f} GB, plan workspaces "
        f"{rp.cost().workspace_bytes / 1e9:.1f} GB")
    cost = rp.cost()
    flops = cost.factor_flops + cost.solve_flops

    def step():
        rp.factor_refine(D, E, C, R, b, x, tol=0.0, max_iters=1)

    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.synchronize()
    graph = None
    if not args.no_graph:
        tc = time.perf_counter()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            step()
        torch.cuda.synchronize()
        log(f"captured the batch solve in {time.perf_counter() - tc:.2f}s")

    def run():
        if graph is not None:
            graph.replay()
        else:
            with torch.cuda.stream(side):
                step()

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - w0) * 1e3)
    info = rp.info()
    err = None
    if not args.no_cpu:
        from oracle import oracle
        worst = 0.0
        for i in sorted({0, K // 3, K // 2, (2 * K) // 3, K - 1}):
            S, N, n, _ = shapes[i]
            host = [rp.unpack(w, t, i).cpu().numpy() for w, t in enumerate((D, E, C, R, b))]
            Dh = host[0].reshape(S, N, n, n)
            Eh = host[1].reshape(S, N - 1, n, n)
            Ch, Rh, bh = host[2].reshape(S, n, n), host[3].reshape(n, n), host[4].reshape(1, -1)
            ref, _ = oracle.solve(Dh, Eh, Ch, Rh, bh, nthreads=host_threads())
            xi = rp.unpack(4, x, i).cpu().numpy().reshape(1, -1)
            worst = max(worst, float(np.max(np.abs(xi - ref)) / np.max(np.abs(ref))))
        err = worst
    ts = sorted(times)
    p50 = statistics.median(ts)
    p99 = ts[min(len(ts) - 1, int(round(0.99 * (len(ts) - 1))))]
    out = {"metric": "batched independent systems, FP32 + 1 refinement correction",
           "value": round(K / (p50 * 1e-3), 1), "unit": "systems/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(p50, 3),
           "p50_ms": round(p50, 3), "p99_ms": round(p99, 3), "higher_is_better": True,
           "dtype": "f32+f64", "data": "synthetic (device generator)",
           "config": {"workload": "c4", "systems": K, "S": "U[8,256]", "N": "U[16,256]",
                      "n": "{8,16,32}", "delta": "log-U[1e-4,1]", "plan": "one ragged plan",
                      "mapping": "autotuned per shape class" if args.tune else "defaults",
                      "padded_work": 1.0, "graph": not args.no_graph},
           "gflops_real_work": round(flops / (p50 * 1e-3) / 1e9, 1),
           "autotuned": tuned or None,
           "input_gb": round(sum(sz) * 8 / 1e9, 1),
           "workspace_gb": round(rp.cost().workspace_bytes / 1e9, 1),
           "info": info, "max_rel_err_vs_oracle_sampled": err}
    print(json.dumps(out))
    rp.close()


def bench_qp(args):
    """IPM front end: assemble the reduced IPM system of a synthetic linear branch-MPC QP
    (S=256 scenarios, N=128 stages, 12 states + 4 inputs, 12 equality and 32
    inequality rows per link) and solve one IPM step with it (FP32 + one refinement
    correction).  One step = assembly + factor + refined solve."""
    import numpy as np
    import torch

    from paper_2609_29977_amd import bmpc
    from synth.qp import make_qp

    S, N, nx, nu = 256, 128, 12, 4
    t0 = time.perf_counter()
    q = make_qp(S, N, nx, nu, tau=1e-6, delta=1e-3, seed=args.seed)
    log(f"generated the QP in {time.perf_counter() - t0:.1f}s")
    n, me, mi = q.n, q.A.shape[2], q.G.shape[2]
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    Q, A, G, w = to(q.Q), to(q.A), to(q.G), to(q.w)
    rng = np.random.default_rng(1)
    b = to(rng.standard_normal((1, (S * N + 1) * n)))
    plan = bmpc.Plan(S, N, n, 1, "fp32")
    x = torch.empty_like(b)
    out_box = {}

    def assemble():
        out_box["K"] = bmpc.assemble_qp(Q, A, G, w, q.tau, q.delta)

    def step():
        assemble()
        D, E, C, R = out_box["K"]
        plan.factor(D, E, C, R)
        plan.refine(D, E, C, R, b, x, tol=0.0, max_iters=1)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    def timed(fn):
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - w0) * 1e3)
        return statistics.median(ts)

    ms_asm = timed(assemble)
    ms_step = timed(step)
    links = S * (N + 1)
    read = links * 8.0 * ((2 * n) ** 2 + (me + mi) * 2 * n + mi)
    written = 8.0 * n * n * (S * N * 2 + S + 1)
    err = None
    if not args.no_cpu:
        from oracle import oracle
        # the dense reduction is too large at this size (the assembly itself is checked
        # against it in the tests): here the refined solve of the assembled system is
        # checked against the oracle's solve of the same blocks
        D, E, C, R = (t.cpu().numpy() for t in out_box["K"])
        ref, info = oracle.solve(D, E, C, R, b.cpu().numpy(), nthreads=16)
        err = float(np.max(np.abs(x.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    out = {"metric": "IPM step: reduced-system assembly + FP32 factor + refined solve",
           "value": round(ms_step, 4), "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": False,
           "dtype": "f64 assembly, f32+f64 solve", "data": "synthetic",
           "config": {"workload": "qp", "S": S, "N": N, "nx": nx, "nu": nu, "me": me, "mi": mi},
           "assembly_ms": round(ms_asm, 4),
           "assembly_gbs": round((read + written) / (ms_asm * 1e-3) / 1e9, 1),
           "rel_err_vs_oracle_solve_of_assembled_system": err}
    print(json.dumps(out))
    plan.close()


def bench_gradients(args):
    """Gradient workload: 64 independent FP64 systems (S=128, N=64, n=16), loss
    0.5 ||x||^2; one step = forward (factor + solve) and backward (adjoint solve +
    block gradients) of every system through the autograd Function."""
    import numpy as np
    import torch

    from paper_2609_29977_amd.autograd import batched_branch_solve
    from synth.branch_system import make_system

    B, S, N, n = 64, 128, 64, 16
    t0 = time.perf_counter()
    systems = [make_system(S, N, n, 1, 1e-2, 100 + i) for i in range(B)]
    log(f"generated {B} systems in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    st = lambda name: torch.from_numpy(np.stack([getattr(s, name) for s in systems])).to(dev)
    D, E, C, R, b = st("D"), st("E"), st("C"), st("R"), st("b")
    params = [D, E, C, R, b]
    for p_ in params:
        p_.requires_grad_()

    def step():
        for p_ in params:
            p_.grad = None
        x = batched_branch_solve(D, E, C, R, b, "fp64")
        (0.5 * (x * x).sum()).backward()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - w0) * 1e3)
    err = None
    if not args.no_cpu:
        from oracle import gradients
        worst = 0.0
        for i in (0, B - 1):
            s = systems[i]
            _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
            for got, ref in ((b.grad[i], db), (D.grad[i], dD), (E.grad[i], dE),
                             (C.grad[i], dC), (R.grad[i], dR)):
                worst = max(worst, float(np.max(np.abs(got.cpu().numpy() - ref)) /
                                         np.max(np.abs(ref))))
        err = worst
    ms = statistics.median(times)
    out = {"metric": "gradient workload: forward+backward of 64 systems (S=128 N=64 n=16, FP64)",
           "value": round(B / (ms * 1e-3), 1), "unit": "systems/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "p99_ms": round(sorted(times)[max(0, int(0.99 * len(times)) - 1)], 4),
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "c5", "systems": B, "S": S, "N": N, "n": n},
           "max_rel_err_vs_oracle_grad": err}
    print(json.dumps(out))


def bench_paper_grid(args):
    """The paper's own workload shape (Section V): n = 16, FP64, one right-hand side, M
    scenarios x N stages on the two lines of its grid that it quotes times for (N = 30
    with M = 20..200, and M = 100 with N = 40..160).  Factor and solve are timed
    separately, each as the median of 50 calls after 10 warm-ups, each call replayed from
    a HIP graph (the paper captures its factor and solve pipelines as graphs).  Seeded
    synthetic systems (delta = 1e-2) stand in for the quadrotor systems."""
    import numpy as np
    import torch

    from paper_2609_29977_amd import bmpc
    from synth.branch_system import make_system

    n, warm, runs = 16, 10, 50
    grid = [(M, 30) for M in range(20, 201, 20)] + [(100, N) for N in range(40, 161, 20)]
    dev = torch.device("cuda:0")
    points, worst = [], 0.0
    for M, N in grid:
        s = make_system(M, N, n, 1, 1e-2, args.seed)
        D, E, C, R, b = (torch.from_numpy(a).to(dev) for a in (s.D, s.E, s.C, s.R, s.b))
        x = torch.empty_like(b)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        p = bmpc.Plan(M, N, n, 1, "fp64", args.window_depth, stream=side)
        with torch.cuda.stream(side):
            p.factor(D, E, C, R)
            p.solve(b, x)
        torch.cuda.synchronize()
        gf, gs = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(gf, stream=side):
            p.factor(D, E, C, R)
        with torch.cuda.graph(gs, stream=side):
            p.solve(b, x)
        torch.cuda.synchronize()

        def med(g):
            for _ in range(warm):
                g.replay()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(runs)]
            for e0, e1 in ev:
                e0.record()
                g.replay()
                e1.record()
            torch.cuda.synchronize()
            return statistics.median(e0.elapsed_time(e1) for e0, e1 in ev)

        tf, ts = med(gf), med(gs)
        gf.replay()
        gs.replay()
        torch.cuda.synchronize()
        if p.info() != 0:
            raise RuntimeError(f"factorization failed at M={M} N={N}")
        if not args.no_cpu:
            from oracle import oracle
            ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=16)
            worst = max(worst, float(np.max(np.abs(x.cpu().numpy() - ref)) /
                                     np.max(np.abs(ref))))
        cost = p.cost()
        points.append({"M": M, "N": N, "factor_ms": round(tf, 4), "solve_ms": round(ts, 4),
                       "factor_gflops": round(cost.factor_flops / (tf * 1e-3) / 1e9, 1)})
        log(f"M={M} N={N}: factor {tf:.4f} ms, solve {ts:.4f} ms")
        p.close()
        del gf, gs
    top = next(q for q in points if q["M"] == 100 and q["N"] == 160)
    out = {"metric": "FP64 factor and solve times on the paper's workload grid (n=16)",
           "value": top["factor_ms"], "unit": "ms", "n_gpus": 1, "steps": runs,
           "warmup": warm, "ms_per_step": round(top["factor_ms"] + top["solve_ms"], 4),
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "paper grid: n=16, N=30 with M=20..200, M=100 with "
                                  "N=40..160; value = factor ms at M=100 N=160",
                      "n": n, "nrhs": 1, "delta": 1e-2, "graph": True},
           "points": points,
           "max_rel_err_vs_oracle": None if args.no_cpu else worst}
    print(json.dumps(out))


FP64_CLASSES = ("root_reduce", "root_potrf", "solve_root", "residual", "residual_root",
                "refine_misc")


def device_copy_rate(torch, mib=1024, reps=10):
    """Read + write GB/s of a plain 1 GiB device copy: the practical streaming ceiling."""
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * (mib << 20) / sec / 1e9


def kernel_rooflines(plan, times, names, fp32, first_pass_extra, copy_gbs):
    """Algorithmic GB/s and TFLOP/s of each kernel class over its measured time per step,
    as fractions of the HBM peak, of the copy rate and of the arithmetic peak."""
    out = {}
    for name, t in times.items():
        bytes_call, flops_call, launches_call = plan.kernel_cost(names.index(name))
        if name == "factor_first_pass":
            bytes_call += first_pass_extra
        sec = t["ms_per_step"] * 1e-3
        if sec <= 0 or (bytes_call <= 0 and flops_call <= 0):
            continue
        calls = t["launches_per_step"] / max(1, launches_call)
        gbs = bytes_call * calls / sec / 1e9
        tfs = flops_call * calls / sec / 1e12
        peak = FP32_MFMA_PEAK_TFS if fp32 and name not in FP64_CLASSES else FP64_PEAK_TFS
        out[name] = {"ms_per_step": round(t["ms_per_step"], 4), "gb_s": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "copy_frac": round(gbs / copy_gbs, 4),
                     "tflop_s": round(tfs, 3), "flop_frac": round(tfs / peak, 4)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the scenario-sharded "
              "multi-GPU path is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy > 0:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
        # factor that turns the counters of the solver kernels into HBM bytes.
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 4}))
        return

    from paper_2609_29977_amd import bmpc
    from synth.branch_system import CONFIGS, make_config

    if args.config == "c5":
        return bench_gradients(args)
    if args.config == "c4":
        return bench_hetero(args)
    if args.config == "qp":
        return bench_qp(args)
    if args.config == "paper":
        return bench_paper_grid(args)

    S, N, n, nrhs, delta = CONFIGS[args.config]
    t0 = time.perf_counter()
    sysd = make_config(args.config, seed=args.seed)
    log(f"generated {args.config} S={S} N={N} n={n} nrhs={nrhs} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)
    D, E, C, R, b = to(sysd.D), to(sysd.E), to(sysd.C), to(sysd.R), to(sysd.b)
    torch.cuda.synchronize()
    names = bmpc.kernel_class_names()

    ta = time.perf_counter()
    p32 = bmpc.Plan(S, N, n, nrhs, "fp32", args.window_depth)
    p64 = bmpc.Plan(S, N, n, nrhs, "fp64", args.window_depth)
    analyze_ms = (time.perf_counter() - ta) * 1e3
    # the same FP32 path with the library deciding when to stop: refinement until the
    # normwise backward error of x, taken from its own FP64 residual, is <= 16 u
    p32c = bmpc.Plan(S, N, n, nrhs, "fp32", args.window_depth)
    p32c.set_refine_stop("backward_error")
    cert_tol = 16 * bmpc.UNIT_ROUNDOFF
    cost = p64.cost()
    flops = cost.factor_flops + cost.solve_flops
    x32 = torch.empty_like(b)
    x64 = torch.empty_like(b)
    x32c = torch.empty_like(b)

    # The timed step: factor + solve with the first solve's forward substitution inside
    # the factorization (bmpc_factor_refine / bmpc_factor_solve); --separate times the
    # separate factor and solve calls instead.  Both are reported.
    def step32_fused():
        p32.factor_refine(D, E, C, R, b, x32, tol=0.0, max_iters=args.ir_steps)

    def step64_fused():
        p64.factor_solve(D, E, C, R, b, x64)

    def step32_sep():
        p32.factor(D, E, C, R)
        p32.refine(D, E, C, R, b, x32, tol=0.0, max_iters=args.ir_steps)

    def step64_sep():
        p64.factor(D, E, C, R)
        p64.solve(b, x64)

    def step32_cert():
        p32c.factor_refine(D, E, C, R, b, x32c, tol=cert_tol, max_iters=10)

    step32, step64 = (step32_sep, step64_sep) if args.separate else (step32_fused, step64_fused)
    alt32, alt64 = (step32_fused, step64_fused) if args.separate else (step32_sep, step64_sep)

    def timed(step, k):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        evs[0].record()
        for i in range(k):
            step()
            evs[i + 1].record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1e3 / k
        per = [evs[i].elapsed_time(evs[i + 1]) for i in range(k)]
        return wall, per

    for _ in range(args.warmup):
        step32()
        step64()
        step32_cert()
    torch.cuda.synchronize()
    log("warmup done")
    ms32, per32 = timed(step32, args.steps)
    ms64, per64 = timed(step64, args.steps)
    ms32c, per32c = timed(step32_cert, args.steps)
    cert_iters, cert_eta, cert_ok = p32c.stats()
    log(f"fp32+ir {ms32:.3f} ms/step, fp64 {ms64:.3f} ms/step, fp32+ir with the backward-error "
        f"stop {ms32c:.3f} ms/step ({cert_iters} corrections, eta {cert_eta:.2e})")
    alt32(), alt64()
    alt_ms32, _ = timed(alt32, args.steps)
    alt_ms64, _ = timed(alt64, args.steps)
    log(f"{'fused' if args.separate else 'separate calls'}: fp32+ir {alt_ms32:.3f} ms/step, "
        f"fp64 {alt_ms64:.3f} ms/step")
    # the timed path's outputs are the ones checked against the oracle
    step32(), step64()

    # Per-kernel times with HIP events recorded by the library on its stream.
    kt = {}
    for tag, plan, step in (("fp32_ir", p32, step32), ("fp64", p64, step64)):
        plan.reset_kernel_times()
        plan.set_profiling(True)
        for _ in range(args.profile_steps):
            step()
        plan.set_profiling(False)
        times = plan.kernel_times()
        kt[tag] = {k: {"launches_per_step": v[0] / args.profile_steps,
                       "ms_per_step": v[1] / args.profile_steps}
                   for k, v in times.items() if v[0] > 0}
    torch.cuda.synchronize()

    # Every kernel class against the HBM peak, the measured copy rate and the peak of
    # the arithmetic it computes in (FP32 for the factor and sweeps of the FP32 path;
    # the residual and the root steps are FP64 in both paths).
    copy_gbs = device_copy_rate(torch)

    def fused_extra(plan, ybytes):
        # with the forward substitution inside, the first pass also reads b (FP64) and
        # writes y for every position it eliminates (all but the multiples of 2^Tw)
        if args.separate:
            return 0.0
        tw = plan.cost().window_depth
        return S * ((N - 1) - (N - 1) // (1 << tw)) * n * nrhs * (8 + ybytes)

    extra32 = fused_extra(p32, 4)
    per_kernel = {"fp32_ir": kernel_rooflines(p32, kt["fp32_ir"], names, True, extra32,
                                              copy_gbs),
                  "fp64": kernel_rooflines(p64, kt["fp64"], names, False,
                                           fused_extra(p64, 8), copy_gbs)}

    # Dominant kernel of the headline path and its roofline.
    dom = max(kt["fp32_ir"].items(), key=lambda kv: kv[1]["ms_per_step"])
    dom_name, dom_t = dom
    cls = names.index(dom_name)
    bytes_call, flops_call, launches_call = p32.kernel_cost(cls)
    if dom_name == "factor_first_pass":
        bytes_call += extra32
    launches = dom_t["launches_per_step"]
    roofline = None
    if bytes_call > 0 and dom_t["ms_per_step"] > 0:
        # average launch of the class: algorithmic bytes of one call spread over the
        # launches of that call, against the measured average launch duration
        per_launch_ms = dom_t["ms_per_step"] / launches
        per_launch_bytes = bytes_call / max(1, launches_call)
        achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
        digest = source_digest(FACTOR_SOURCES if dom_name.startswith("factor_") else None)
        traffic = measured_traffic(dom_name + ":fp32", digest)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "kernel": dom_name,
                    "bytes_per_launch": per_launch_bytes, "ms_per_launch": per_launch_ms,
                    "flops_per_launch": flops_call / max(1, launches_call),
                    "achieved_tflops": round(flops_call / max(1, launches_call) /
                                             (per_launch_ms * 1e-3) / 1e12, 3),
                    "source_digest": digest}

    # Accuracy against the FP64 oracle and the CPU baseline (oracle timed on the host).
    err32 = err64 = err32c = None
    cpu = None
    kappa = None
    iters, relc, _ = p32.stats()
    if not args.no_cpu:
        from oracle import oracle
        ref, info, (tf, ts) = oracle.solve(sysd.D, sysd.E, sysd.C, sysd.R, sysd.b,
                                           nthreads=host_threads(), return_times=True)
        scale = float(np.max(np.abs(ref)))
        err32 = float(np.max(np.abs(x32.cpu().numpy() - ref)) / scale)
        err64 = float(np.max(np.abs(x64.cpu().numpy() - ref)) / scale)
        err32c = float(np.max(np.abs(x32c.cpu().numpy() - ref)) / scale)
        log(f"oracle on the whole system {tf + ts:.2f}s; err fp32+ir {err32:.2e} fp64 "
            f"{err64:.2e} certified {err32c:.2e}")
        cpu = cpu_baseline(sysd, args.config)
        kappa = measured_kappa(args.config)
    gfs32 = flops / (ms32 * 1e-3) / 1e9
    gfs64 = flops / (ms64 * 1e-3) / 1e9
    out = {
        "metric": "factor+solve µs & GFLOP/s, S=512 N=256 n=32: FP32+IR vs FP64 at rel err 1e-10",
        "value": round(gfs32, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: S={S} N={N} n={n} nrhs={nrhs} delta={delta}, "
                               f"FP32 factor+solve + {args.ir_steps} FP64-residual refinement step"
                               + ("" if args.separate else
                                  "; first forward substitution inside the factorization"),
                   "S": S, "N": N, "n": n, "nrhs": nrhs, "seed": args.seed,
                   "window_depth": p32.cost().window_depth},
        "fp32_ir": {"ms_per_step": round(ms32, 4), "median_ms": round(statistics.median(per32), 4),
                    "gflops": round(gfs32, 2), "rel_err_vs_oracle": err32,
                    "ir_corrections": iters, "last_rel_correction": relc,
                    "kernels_ms_per_step": {k: round(v["ms_per_step"], 4)
                                            for k, v in kt["fp32_ir"].items()}},
        "fp32_ir_certified": {
            "ms_per_step": round(ms32c, 4), "median_ms": round(statistics.median(per32c), 4),
            "gflops": round(flops / (ms32c * 1e-3) / 1e9, 2), "rel_err_vs_oracle": err32c,
            "stop": "normwise backward error <= 16u from the FP64 residual of the returned x",
            "ir_corrections": cert_iters, "backward_error": cert_eta, "converged": cert_ok,
            "speedup_vs_fp64": round(ms64 / ms32c, 3)},
        "fp64": {"ms_per_step": round(ms64, 4), "median_ms": round(statistics.median(per64), 4),
                 "gflops": round(gfs64, 2), "rel_err_vs_oracle": err64,
                 "kernels_ms_per_step": {k: round(v["ms_per_step"], 4)
                                         for k, v in kt["fp64"].items()}},
        "fp32_ir_speedup_vs_fp64": round(ms64 / ms32, 3),
        "forward_in_factor": not args.separate,
        ("fused" if args.separate else "separate_calls"): {
            "fp32_ir_ms_per_step": round(alt_ms32, 4), "fp64_ms_per_step": round(alt_ms64, 4)},
        "method_flops_per_step": flops,
        "analyze_ms": round(analyze_ms, 2),
        "roofline": roofline,
        "copy_gb_s": round(copy_gbs, 1),
        "kernels_roofline": per_kernel,
        "cpu_baseline": cpu,
        "kappa": kappa,
    }
    print(json.dumps(out), flush=True)
    p32.close()
    p64.close()
    p32c.close()


def host_threads():
    """Threads the oracle may use: the CPU affinity of this process, at most 16 (the
    host's CPU share for one GPU)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sysd, config):
    """The oracle (natural-order band Cholesky + solve, FP64, OpenMP over scenarios)
    timed on this host: single-threaded and on every thread of the host's share, each
    the median of 3 runs after 1 warm-up, on a bounded sample of the workload (the
    first scenarios of the system, all stages, its root block); the oracle's work is
    linear in the scenarios, so the rate holds for the whole system."""
    import numpy as np

    from oracle import oracle
    from paper_2609_29977_amd import bmpc

    S, N, n = sysd.S, sysd.N, sysd.n

    def sample(Ss):
        Ss = min(S, Ss)
        b = np.concatenate([sysd.b[:, :Ss * N * n], sysd.b[:, S * N * n:]], axis=1)
        c = bmpc.cost_model(Ss, N, n, sysd.nrhs, "fp64")
        return (sysd.D[:Ss], sysd.E[:Ss], sysd.C[:Ss], sysd.R, b), Ss, c.factor_flops + c.solve_flops

    def med(args, threads):
        ts = []
        for _ in range(4):
            _, _, (tf, tsol) = oracle.solve(*args, nthreads=threads, return_times=True)
            ts.append(tf + tsol)
        return statistics.median(ts[1:])

    threads = host_threads()
    used = oracle.threads_used(threads)
    args1, s1, fl1 = sample(max(1, S // 32))
    t1 = med(args1, 1)
    argsT, sT, flT = sample(max(1, S // 8))
    tT = med(argsT, threads)
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"value": round(flT / tT / 1e9, 3), "unit": "GFLOP/s", "cores": used,
            "kind": "oracle",
            "sample": f"{config} with its first {sT} of {S} scenarios (all {N} stages, "
                      f"n={n}, root block), one factor+solve, median of 3 after 1: "
                      f"{tT * 1e3:.0f} ms on {used} threads; natural-order band Cholesky, "
                      "OpenMP over scenarios",
            "single_thread": {"value": round(fl1 / t1 / 1e9, 3), "unit": "GFLOP/s",
                              "sample_scenarios": s1, "ms": round(t1 * 1e3, 1),
                              "est_full_system_s": round(t1 * S / s1, 1)},
            "all_threads": {"value": round(flT / tT / 1e9, 3), "threads": used,
                            "sample_scenarios": sT, "ms": round(tT * 1e3, 1),
                            "est_full_system_s": round(tT * S / sT, 2)},
            "cpu_model": cpu_model(), "host_cpus": nproc, "os_cpu_count": os.cpu_count(),
            "thread_cap": "16 = the host's CPU share for one GPU"}


def measured_kappa(config):
    """kappa(K) = lambda_max / lambda_min of the workload's generator on a copy with 8
    stages (same S, n, delta, seed; kappa is set by S, not N), by Lanczos and
    shift-invert Lanczos (oracle.conditioning)."""
    from oracle.conditioning import extreme_eigenvalues
    from synth.branch_system import CONFIGS, make_system
    S, N, n, nrhs, delta = CONFIGS[config]
    Nk = min(N, 8)
    s = make_system(S, Nk, n, 1, delta, 0)
    t0 = time.perf_counter()
    lmin, lmax = extreme_eigenvalues(s.D, s.E, s.C, s.R)
    return {"value": round(lmax / lmin, 1), "lambda_min": lmin, "lambda_max": lmax,
            "measured_on": f"{config} generator with N={Nk} (S={S}, n={n}, delta={delta}, seed 0)",
            "seconds": round(time.perf_counter() - t0, 1)}


if __name__ == "__main__":
    main()
