#!/usr/bin/env python3
"""Benchmark of the sparse Tucker hot path on one GPU.

Workload (default): sparse 1000 x 1000 x 1000 tensor with 1,000,000
uniformly random distinct nonzeros, values U(0,1) (seeded, synthetic), core
50 x 50 x 50, Multislice Projection, 10 sweeps, BF16 Grams with FP32
accumulation and FP64 eigensolve / core / fit. One step = one complete
decomposition (validation, orderings, HO-SVD start, 10 sweeps) with the
tensor already resident in HBM.

The JSON line reports:
* value: projected nonzeros per second over the TTMc phase of the sweeps
  (every projection launch projects all nonzeros onto one factor; the sum of
  their HIP-event times is the TTMc phase), median over the timed steps;
* time-to-fit of plain FP32 vs mixed BF16 runs that stop on the paper's
  Delta-fit < 1e-4 rule;
* roofline of the projection kernel, the metric's kernel (live HIP-event
  times on the library's stream x algorithmic bytes per launch), and of the
  Gram kernel beside it (algorithmic flops per launch);
* parity_small: every precision form against the FP64 oracle's stored
  numbers on the small workload (fit differences, factor subspace angles);
* cpu_baseline: one sweep of the FP64 oracle on the host cores, same input.
"""
import argparse
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
METRIC = "projected nnz/s per TTMc sweep + time-to-fit (|Δfit|≤1e-4) mixed vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def project_bytes(nnz, nslots, J, I_m, precision):
    """Bytes one projection launch must move: leaf index + value per nonzero
    (FP64 values for fp64, else FP32), slot pointers, the dense projected
    tensor, the factor copy it reads (FP16 rows for mixed)."""
    out_bytes = {"mixed": 2, "fp32": 4, "fp64": 8}[precision]
    val_bytes = 8 if precision == "fp64" else 4
    fac_bytes = {"mixed": 2, "fp32": 4, "fp64": 8}[precision]
    return nnz * (4 + val_bytes) + (nslots + 1) * 4 + nslots * J * out_bytes + I_m * J * fac_bytes


def gram_flops(I, J, n):
    """Useful flops of the MP Gram of mode n: both projected terms, lower
    triangle with diagonal, multiply+add = 2 flops."""
    total = 0
    for m in range(3):
        if m == n:
            continue
        K = (I[0] * I[1] * I[2] // (I[n] * I[m])) * J[m]
        total += I[n] * (I[n] + 1) * K
    return total


def traffic_from_profile(kernel_file):
    """HBM bytes per launch of the projection kernel measured by rocprofv3
    counters, if the committed measurement matches the current source."""
    path = os.path.join(ROOT, "profiles", "k_project_mixed_1000cube_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    with open(kernel_file, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    if d.get("source_sha256") != h:
        return None
    return d.get("bytes_per_launch")


def subspace_angle(A, B):
    """Largest principal angle between span(A) and span(B) (orthonormal
    columns): arcsin of the spectral norm of B's part outside span(A), the
    form that stays accurate at small angles. The comparison the benchmark
    reports; a CPU test holds it equal to the oracle's."""
    import numpy as np
    R = B - A @ (A.T @ B)
    return float(np.arcsin(min(1.0, np.linalg.norm(R, 2))))


def learned_model(tk, dev):
    """Train the learned start's network on the GPU from the generator
    tensors and the oracle-converged factors stored with the tests (written
    by tests/golden/make_learn_targets.py, which runs the oracle only)."""
    import numpy as np
    import torch
    import synth
    from paper_0711_2023_amd import learn as TL
    d = np.load(os.path.join(ROOT, "tests", "golden", "learn_targets.npz"), allow_pickle=False)
    samples = []
    for k, r in enumerate(d["recipes"]):
        kind, I1, I2, I3, J1, J2, J3, nnz, seed, noise, held = r
        if held:
            continue
        dims, core = (int(I1), int(I2), int(I3)), (int(J1), int(J2), int(J3))
        if int(kind) == 0:
            idx, vals, dims = synth.planted_tucker(dims, core, int(nnz), float(noise), int(seed))
        else:
            idx, vals, dims = synth.uniform_sparse(dims, int(nnz), int(seed))
        di = torch.from_numpy(idx.astype(np.int32)).to(dev)
        dv = torch.from_numpy(vals).to(dev)
        for mode in (1, 2):
            samples.append(TL.make_sample(di, dv, dims, mode, d[f"t{k}_m{mode}"]))
    params = TL.init_params(3, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = TL.train(params, samples, steps=600, lr=2e-3)
    torch.cuda.synchronize()
    info = {"samples": len(samples), "steps": 600, "seconds": round(time.perf_counter() - t0, 3),
            "loss_first_pass": round(float(np.mean(losses[:len(samples)])), 4),
            "loss_last_pass": round(float(np.mean(losses[-len(samples):])), 4)}
    return params, info


def learned_leg(args):
    """Time-to-fit of the mixed run started from the learned start (the
    network trained first, not timed), printed as one JSON line."""
    import numpy as np
    import torch
    import paper_0711_2023_amd as tk
    import synth
    tk.lib()
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[args.workload]
    dims, J, nnz = tuple(w["dims"]), tuple(w["core"]), int(w["nnz"])
    idx, vals, dims = synth.uniform_sparse(dims, nnz, w["seed"])
    di = torch.from_numpy(idx.astype(np.int32)).to(dev)
    dv = torch.from_numpy(vals).to(dev)
    fn = tk.mp if args.algo == "mp" else tk.hooi
    log("learned leg: training")
    model, info = learned_model(tk, dev)
    log(f"learned leg: trained {info}")
    runs = []
    for k in range(3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = fn(di, dv, dims, J, precision="mixed", max_iters=50, tol=1e-4, init=tk.INIT_LEARNED, model=model)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t1, r))
        log(f"learned leg: run {k} {1000 * runs[-1][0]:.1f} ms, {r.iters} sweeps, fit {r.fits[-1]:.6e}")
    runs.sort(key=lambda x: x[0])
    tw, r = runs[1]
    print(json.dumps({"wall_ms": round(1000 * tw, 2), "sweeps": r.iters, "fit": r.fits[-1],
                      "prep_excluded_ms": round(r.stats["init_ms"] + r.stats["sweeps_ms"], 2),
                      "init_ms": round(r.stats["init_ms"], 2), "init_fallbacks": r.stats["init_fallbacks"],
                      "training": info}), flush=True)
    return 0


def batched_leg(tk, dev, sweeps):
    """64 tensors (mode sizes U{200..800}, density 0.5 %, cores U{10..40},
    U(0,1) values), MP with BF16 Grams, `sweeps` sweeps each: one call on 8
    streams against the same call on one stream, and the 8-stream call again
    with the tuner's launch choices per shape bucket."""
    import numpy as np
    import torch
    import synth
    cfgs = synth.batch_configs(64, 3000)
    tensors, cores, total = [], [], 0
    for c in cfgs:
        idx, vals, dims = synth.uniform_sparse(c["dims"], c["nnz"], c["seed"])
        tensors.append((torch.from_numpy(idx.astype(np.int32)).to(dev), torch.from_numpy(vals).to(dev), dims))
        cores.append(c["core"])
        total += c["nnz"]
    out = {"workload": "64 sparse tensors, mode sizes U{200..800}, density 0.5 %, cores U{10..40}, U(0,1) values, "
                       f"MP mixed, {sweeps} sweeps each", "tensors": 64, "nnz_total": total}
    for ns in (8, 1):
        streams = [torch.cuda.Stream(device=dev) for _ in range(ns)]
        tk.batched(tk.ALGO_MP, tensors[:ns], cores[:ns], streams=streams, precision="mixed", max_iters=2, tol=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, st = tk.batched(tk.ALGO_MP, tensors, cores, streams=streams, precision="mixed", max_iters=sweeps,
                             tol=0.0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[f"wall_ms_{ns}_streams"] = round(1000 * wall, 1)
        out[f"tensors_per_s_{ns}_streams"] = round(64 / wall, 2)
        out[f"swept_nnz_per_s_{ns}_streams"] = round(total * sweeps / wall, 1)
        log(f"batched: {ns} stream(s) {1000 * wall:.1f} ms for 64 tensors")
    out["speedup_8_over_1_stream"] = round(out["wall_ms_1_streams"] / out["wall_ms_8_streams"], 3)
    # launch choices per shape bucket from the tuner (measured before the
    # timed call; results within rounding of the built-in choices)
    from paper_0711_2023_amd import autotune
    t0 = time.perf_counter()
    cache = autotune.TuneCache()
    tunes = autotune.tune_batch(tk.ALGO_MP, tensors, cores, "mixed", cache, reps=1)
    out["tune_s"] = round(time.perf_counter() - t0, 2)
    out["tune_buckets"] = len(cache.entries)
    out["tuned_choices"] = sorted({str(t.key()) for t in tunes})
    streams = [torch.cuda.Stream(device=dev) for _ in range(8)]
    tk.batched(tk.ALGO_MP, tensors[:8], cores[:8], streams=streams, tunes=tunes[:8], precision="mixed",
               max_iters=2, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tk.batched(tk.ALGO_MP, tensors, cores, streams=streams, tunes=tunes, precision="mixed", max_iters=sweeps,
               tol=0.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["wall_ms_8_streams_tuned"] = round(1000 * wall, 1)
    log(f"batched: 8 streams with tuned launch choices {1000 * wall:.1f} ms (tuning {out['tune_s']} s)")
    return out


def parity_leg(tk, dev):
    """Every precision form of MP and HOOI (10 sweeps, HO-SVD start) on two small
    seeded tensors -- the uniform workload (100^3, 10,000 nonzeros, core 10^3)
    and a planted Tucker model of that shape (100,000 entries, noise 0.1) --
    against the FP64 oracle's numbers stored in tests/golden/small_reference.npz
    (written by tests/golden/make_small_reference.py; the oracle is not run
    here): the largest |fit difference| over the sweeps and the largest
    principal angle between GPU and oracle factor subspaces over the modes."""
    import numpy as np
    import torch
    import synth
    ref = np.load(os.path.join(ROOT, "tests", "golden", "small_reference.npz"), allow_pickle=False)

    out = {"reference": "FP64 oracle (stored)", "sweeps": 10, "start": "HO-SVD"}
    for case in ("uniform", "planted"):
        dims = tuple(int(x) for x in ref[f"{case}_dims"])
        J = tuple(int(x) for x in ref[f"{case}_core"])
        nnz, seed = int(ref[f"{case}_nnz"]), int(ref[f"{case}_seed"])
        if case == "uniform":
            idx, vals, dims = synth.uniform_sparse(dims, nnz, seed)
        else:
            idx, vals, dims = synth.planted_tucker(dims, J, nnz, float(ref["planted_noise"]), seed)
        di = torch.from_numpy(idx.astype(np.int32)).to(dev)
        dv = torch.from_numpy(vals).to(dev)
        res = {"tensor": f"{dims[0]}x{dims[1]}x{dims[2]}, {nnz} nonzeros, core {J[0]}x{J[1]}x{J[2]}"}
        for algo in ("mp", "hooi"):
            fo = ref[f"{case}_{algo}_fits"]
            for prec in ("fp64", "fp32", "mixed") + (("bf16x3",) if algo == "mp" else ()):
                r = getattr(tk, algo)(di, dv, dims, J, precision=prec, max_iters=len(fo), tol=0.0)
                fg = np.array(r.fits)
                ang = max(subspace_angle(ref[f"{case}_{algo}_{k}"], f.cpu().numpy()) for k, f in zip("ABC", r.factors))
                res[f"{algo}_{prec}"] = {"max_abs_fit_diff": float(np.max(np.abs(fg - fo))),
                                         "max_subspace_angle_rad": ang}
        out[case] = res
    return out


def cpu_baseline(idx, vals, dims, J, sweeps=1):
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    X = O.SparseTensor3(idx, vals, dims)
    rng = np.random.default_rng(11)
    B0 = np.linalg.qr(rng.standard_normal((dims[1], J[1])))[0]
    C0 = np.linalg.qr(rng.standard_normal((dims[2], J[2])))[0]
    t0 = time.perf_counter()
    O.mp(X, J, sweeps, 0.0, init=(None, B0, C0))
    dt = time.perf_counter() - t0
    return {"value": 3 * X.nnz * sweeps / dt, "unit": "nnz/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{sweeps} full sweep(s) of the FP64 oracle's Multislice Projection (slice-wise Grams, "
                      f"eigendecomposition of M M^T, slice-wise core and fit) on the same input; "
                      f"3*nnz*sweeps / wall time; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube1000_nnz1m")
    ap.add_argument("--algo", default="mp", choices=["mp", "hooi"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--sweeps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-ttf", action="store_true", help="skip the time-to-fit runs")
    ap.add_argument("--no-learn", action="store_true", help="skip the learned-start leg of the time-to-fit runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-tensor leg")
    ap.add_argument("--learned-leg", action="store_true",
                    help="internal: train the learned start, time the mixed run from it, print one JSON line")
    ap.add_argument("--no-parity", action="store_true", help="skip the small-workload comparison with the "
                    "stored oracle reference")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration for profiles)")
    args = ap.parse_args()
    if args.learned_leg:
        return learned_leg(args)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0711_2023_amd as tk
    import synth

    tk.lib()  # fail loudly if the HIP library is missing
    w = synth.WORKLOADS[args.workload]
    dims, J, nnz = tuple(w["dims"]), tuple(w["core"]), int(w["nnz"])
    log(f"generating {args.workload}: dims {dims} nnz {nnz} core {J}")
    idx, vals, dims = synth.uniform_sparse(dims, nnz, w["seed"])
    dev = torch.device("cuda:0")
    di = torch.from_numpy(idx).to(dev)
    dv = torch.from_numpy(vals).to(dev)
    fn = tk.mp if args.algo == "mp" else tk.hooi
    algo_id = tk.ALGO_MP if args.algo == "mp" else tk.ALGO_HOOI
    # one workspace large enough for every precision the legs below run
    precs = [args.precision, "fp32", "mixed"] + (["bf16x3"] if args.algo == "mp" else [])
    wsb = max(tk.workspace_bytes(algo_id, di, dv, dims, J, precision=pr) for pr in precs)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    log(f"workspace {wsb / 2**30:.2f} GiB")

    if args.copy_calib:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration done (3 x 1 GiB)")

    def step(prec, sweeps, tol):
        return fn(di, dv, dims, J, precision=prec, max_iters=sweeps, tol=tol, timing=True, workspace=ws)

    for i in range(args.warmup):
        r = step(args.precision, args.sweeps, 0.0)
        log(f"warmup {i}: fits {r.fits[-1]:.6e} sweeps_ms {r.stats['sweeps_ms']:.1f}")
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step(args.precision, args.sweeps, 0.0)
        results.append(r)
        log(f"step {i}: fit {r.fits[-1]:.6e} prep {r.stats['prep_ms']:.1f} init {r.stats['init_ms']:.1f} "
            f"sweeps {r.stats['sweeps_ms']:.1f} ms (proj {r.stats['project_ms']:.2f}, gram {r.stats['gram_ms']:.2f}, "
            f"eig {r.stats['eig_ms']:.2f}, core {r.stats['core_ms']:.2f})")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / max(1, args.steps)

    nu = results[0].stats["nnz_unique"]
    if args.algo == "mp":
        # every MP projection launch projects all nonzeros onto one factor
        rates = [r.stats["project_calls"] * nu / (r.stats["ttmc_ms"] / 1000.0) for r in results]
    else:
        # a HOOI sweep projects the nonzeros onto all three factors (two
        # projections plus three second-stage GEMMs)
        rates = [3 * nu * r.iters / (r.stats["ttmc_ms"] / 1000.0) for r in results]
    value = statistics.median(rates)
    st = results[len(results) // 2].stats
    sweeps = results[0].iters
    # per-launch averages
    proj_ms = st["project_ms"] / max(1, st["project_calls"])
    gram_ms = st["gram_ms"] / max(1, st["gram_calls"])
    nslots = [dims[(m + 2) % 3] * dims[(m + 1) % 3] for m in range(3)]
    pbytes = statistics.mean(project_bytes(nu, nslots[m], J[m], dims[m], args.precision) for m in range(3))
    proj_gbs = pbytes / (proj_ms / 1000.0) / 1e9
    gflops = statistics.mean(gram_flops(dims, J, n) for n in range(3))
    gram_tf = gflops / (gram_ms / 1000.0) / 1e12
    gpeak = PEAK_TFLOPS["bf16" if args.precision == "mixed" else args.precision]
    kfile = os.path.join(ROOT, "paper_0711_2023_amd", "csrc", "project.hip")
    traffic = traffic_from_profile(kfile)
    roof_proj = {"kernel": "k_project", "bound": "hbm", "achieved": round(proj_gbs, 1), "peak": PEAK_HBM_GBS,
                 "unit": "GB/s", "frac": round(proj_gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
                 "algorithmic_bytes_per_launch": int(pbytes), "avg_launch_ms": round(proj_ms, 5)}
    roof_gram = {"kernel": "k_gram", "bound": "mfma", "achieved": round(gram_tf, 2), "peak": gpeak,
                 "unit": "TFLOP/s", "frac": round(gram_tf / gpeak, 4), "traffic": None,
                 "algorithmic_flops_per_launch": int(gflops), "avg_launch_ms": round(gram_ms, 5)}
    # the roofline line is the kernel of the metric (the projection); the
    # Gram's MFMA fraction goes beside it
    dominant, other = roof_proj, (roof_gram if args.algo == "mp" else None)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "bf16(gram)+fp32(proj,acc)+fp64(eig,core,fit)", "fp32": "fp32+fp64(eig,core,fit)",
                  "fp64": "fp64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"sparse {dims[0]}x{dims[1]}x{dims[2]}, {nnz} uniform distinct nonzeros, U(0,1) "
                               f"values, core {J[0]}x{J[1]}x{J[2]}, {args.algo.upper()}, {args.sweeps} sweeps",
                   "dims": list(dims), "nnz": nnz, "core": list(J), "algo": args.algo,
                   "precision": args.precision, "sweeps": sweeps, "seed": w["seed"]},
        "roofline": dominant,
        "phase_ms_per_sweep": {k: round(st[k] / max(1, sweeps), 4) for k in
                               ("project_ms", "ttmc_ms", "gram_ms", "eig_ms", "core_ms")},
        "whole_sweep_nnz_per_s": 3 * nu / (st["sweeps_ms"] / 1000.0 / max(1, sweeps)),
        "prep_ms": round(st["prep_ms"], 3),
        "init_ms": round(st["init_ms"], 3),
        "fit": results[0].fits[-1],
    }
    if other is not None:
        line["roofline_other"] = other

    if not args.no_ttf:
        ttf = {}
        for prec in ("fp32", "mixed") + (("bf16x3",) if args.algo == "mp" else ()):
            runs = []
            for _ in range(3):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                r = fn(di, dv, dims, J, precision=prec, max_iters=50, tol=1e-4, workspace=ws)
                torch.cuda.synchronize()
                runs.append((time.perf_counter() - t1, r))
            runs.sort(key=lambda x: x[0])
            tw, r = runs[1]
            ttf[prec] = {"wall_ms": round(1000 * tw, 2), "sweeps": r.iters, "fit": r.fits[-1],
                         "prep_excluded_ms": round(r.stats["init_ms"] + r.stats["sweeps_ms"], 2)}
            log(f"time-to-fit {prec}: {ttf[prec]}")
        ttf["speedup_plain_over_mixed"] = round(ttf["fp32"]["wall_ms"] / ttf["mixed"]["wall_ms"], 3)
        ttf["mixed_reaches_plain_fit"] = bool(ttf["mixed"]["fit"] >= ttf["fp32"]["fit"] - 1e-4)
        if "bf16x3" in ttf:  # split-BF16 Grams: FP32-like accuracy
            ttf["speedup_plain_over_bf16x3"] = round(ttf["fp32"]["wall_ms"] / ttf["bf16x3"]["wall_ms"], 3)
        if not args.no_learn:
            # in a child process with a time limit, so that this line is
            # printed whatever happens there
            cmd = [sys.executable, os.path.abspath(__file__), "--learned-leg", "--workload", args.workload,
                   "--algo", args.algo]
            try:
                # progress lines of the child go straight to this process's stderr
                r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=300)
                leg = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 and r.stdout.strip() \
                    else {"error": f"exit {r.returncode}"}
            except subprocess.TimeoutExpired:
                leg = {"error": "timed out after 300 s"}
            ttf["mixed_learned"] = leg
            if "wall_ms" in leg:
                ttf["speedup_plain_over_mixed_learned"] = round(ttf["fp32"]["wall_ms"] / leg["wall_ms"], 3)
                ttf["mixed_learned_reaches_plain_fit"] = bool(leg["fit"] >= ttf["fp32"]["fit"] - 1e-4)
        line["time_to_fit"] = ttf

    if not args.no_batch:
        line["batched"] = batched_leg(tk, dev, args.sweeps)

    if not args.no_parity:
        line["parity_small"] = parity_leg(tk, dev)
        log(f"parity against the stored FP64 oracle reference: {line['parity_small']}")

    if not args.no_cpu:
        log("timing the FP64 oracle (one sweep) on the host")
        line["cpu_baseline"] = cpu_baseline(idx, vals, dims, J, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    sys.exit(main() or 0)
